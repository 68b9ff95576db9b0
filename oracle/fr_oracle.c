/*
 * fr_oracle.c -- plain FP64 CPU oracle of the impact-based fair ranking solver
 * (Uehara et al., "Fast solution to the fair ranking problem using the Sinkhorn
 * algorithm").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference
 * against which the GPU library is checked.  It shares no code, header, table or
 * helper with the GPU path; only the test suite, the package's smoke check and
 * the benchmark's CPU-baseline leg may load it.
 *
 * Everything is double precision, written in the textbook form of each step:
 *
 *   problem (Section 2):  X_u in R^{I x m}; rows sum to 1 (Eq. dsm1); columns
 *       k < m sum to 1 (Eq. dsm2); x >= 0 (Eq. dsm4); the last column is the
 *       dummy position, whose column sums to I - m + 1.
 *   impact (Eq. Imp):     Imp_i = sum_u sum_{k<m} r(u,i) e(k) x_uik.
 *   objective (Eq. objF): F = sum_i log Imp_i.
 *   entropic OT (problem otp, Section 3) solved by log-domain Sinkhorn, cold
 *       start g = 0, T full iterations of (row half-step, column half-step):
 *         f_i = -eps * LSE_k((g_k - c_ik)/eps)
 *         g_k =  eps * log b_k - eps * LSE_i((f_i - c_ik)/eps)
 *       and X = exp((f_i + g_k - c_ik)/eps).  Every LSE is evaluated with its
 *       own max shift; two exponentials per cell and iteration.
 *   gradient (Section 3, "chain rule"): reverse mode through the T stored
 *       iterates of the recursion above.
 *   Algorithm 1: ascent on C with Adam (Section 4.1 names PyTorch's Adam) or
 *       plain gradient ascent.
 *
 * Parallelism: OpenMP over consumers (the only independent axis the paper
 * names: "for u in U do in parallel").  Reductions over consumers are done
 * serially in consumer order.
 *
 * All functions return 0 on success and a negative number on an argument or
 * allocation error.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_EXPORT __attribute__((visibility("default")))

/* Column mass b_k of the transportation polytope: 1 for the m-1 real
 * positions (Eq. dsm2), I - m + 1 for the dummy (text after Eq. dsm4).
 * k is 0-based, so the dummy is k = m-1. */
static double col_mass(int k, int I, int m) {
    return (k < m - 1) ? 1.0 : (double)(I - m + 1);
}

/* log-sum-exp of n values spaced by `stride` */
static double lse(const double* z, int n, int stride) {
    double mx = -INFINITY;
    for (int j = 0; j < n; ++j) {
        double v = z[(size_t)j * stride];
        if (v > mx) mx = v;
    }
    if (mx == -INFINITY) return -INFINITY;
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += exp(z[(size_t)j * stride] - mx);
    return mx + log(s);
}

static int check_shape(int64_t U, int I, int m) {
    if (U < 1 || I < 2 || m < 2 || m > I) return -1;
    return 0;
}

/* One full Sinkhorn iteration for one consumer: row half-step from g, then
 * column half-step from the new f.  z is scratch of max(I, m) doubles. */
static void sinkhorn_iter(int I, int m, const double* c, double eps,
                          double* f, double* g, double* z) {
    for (int i = 0; i < I; ++i) {
        for (int k = 0; k < m; ++k) z[k] = (g[k] - c[(size_t)i * m + k]) / eps;
        f[i] = -eps * lse(z, m, 1);
    }
    for (int k = 0; k < m; ++k) {
        for (int i = 0; i < I; ++i) z[i] = (f[i] - c[(size_t)i * m + k]) / eps;
        g[k] = eps * log(col_mass(k, I, m)) - eps * lse(z, I, 1);
    }
}

/* Sinkhorn for one consumer, T iterations from g = 0.  Optional histories:
 * fh [T][I] holds f^1..f^T, gh [T+1][m] holds g^0..g^T. */
static void sinkhorn_one(int I, int m, const double* c, double eps, int T,
                         double* f, double* g, double* z, double* fh, double* gh) {
    for (int k = 0; k < m; ++k) g[k] = 0.0;
    for (int i = 0; i < I; ++i) f[i] = 0.0;
    if (gh) memcpy(gh, g, sizeof(double) * m);
    for (int t = 1; t <= T; ++t) {
        sinkhorn_iter(I, m, c, eps, f, g, z);
        if (fh) memcpy(fh + (size_t)(t - 1) * I, f, sizeof(double) * I);
        if (gh) memcpy(gh + (size_t)t * m, g, sizeof(double) * m);
    }
}

static void plan_from_potentials(int I, int m, const double* c, double eps,
                                 const double* f, const double* g, double* X) {
    for (int i = 0; i < I; ++i)
        for (int k = 0; k < m; ++k)
            X[(size_t)i * m + k] = exp((f[i] + g[k] - c[(size_t)i * m + k]) / eps);
}

/* ------------------------------------------------------------------------ */
/* Forward: X_u = Sinkhorn_T(C_u) for every consumer.  X [U][I][m], f [U][I],
 * g [U][m]; each output may be NULL. */
ORC_EXPORT int fro_forward(int64_t U, int I, int m, const double* C, double eps, int T,
                           double* X, double* f_out, double* g_out) {
    if (check_shape(U, I, m) || !(eps > 0) || T < 1 || !C) return -1;
    int err = 0;
#pragma omp parallel
    {
        double* f = (double*)malloc(sizeof(double) * I);
        double* g = (double*)malloc(sizeof(double) * m);
        double* z = (double*)malloc(sizeof(double) * (I > m ? I : m));
        if (!f || !g || !z) {
#pragma omp atomic write
            err = -2;
        } else {
#pragma omp for schedule(static)
            for (int64_t u = 0; u < U; ++u) {
                const double* c = C + (size_t)u * I * m;
                sinkhorn_one(I, m, c, eps, T, f, g, z, NULL, NULL);
                if (X) plan_from_potentials(I, m, c, eps, f, g, X + (size_t)u * I * m);
                if (f_out) memcpy(f_out + (size_t)u * I, f, sizeof(double) * I);
                if (g_out) memcpy(g_out + (size_t)u * m, g, sizeof(double) * m);
            }
        }
        free(f); free(g); free(z);
    }
    return err;
}

/* Warm-started forward: for each consumer, iterate from the column
 * potentials g_io[u] (in/out, [U][m]) until the column half-step changes no
 * potential by more than tol in log2 units (max_k |g^t_k - g^{t-1}_k| /
 * (eps ln 2) <= tol), or T_max iterations; tol = 0 runs exactly T_max.
 * X from the final potentials; iters_out[u] = iterations used (optional),
 * f_out [U][I] (optional). */
ORC_EXPORT int fro_forward_warm(int64_t U, int I, int m, const double* C, double eps,
                                double* g_io, double tol, int T_max, double* X, double* f_out,
                                int* iters_out) {
    if (check_shape(U, I, m) || !(eps > 0) || T_max < 1 || !C || !g_io || !X) return -1;
    int err = 0;
    const double to_log2 = 1.0 / (eps * log(2.0));
#pragma omp parallel
    {
        double* f = (double*)malloc(sizeof(double) * I);
        double* gp = (double*)malloc(sizeof(double) * m);
        double* z = (double*)malloc(sizeof(double) * (I > m ? I : m));
        if (!f || !gp || !z) {
#pragma omp atomic write
            err = -2;
        } else {
#pragma omp for schedule(static)
            for (int64_t u = 0; u < U; ++u) {
                const double* c = C + (size_t)u * I * m;
                double* g = g_io + (size_t)u * m;
                int t = 0;
                for (t = 1; t <= T_max; ++t) {
                    memcpy(gp, g, sizeof(double) * m);
                    sinkhorn_iter(I, m, c, eps, f, g, z);
                    double worst = 0.0;
                    for (int k = 0; k < m; ++k) {
                        const double d = fabs(g[k] - gp[k]) * to_log2;
                        if (d > worst) worst = d;
                    }
                    if (tol > 0.0 && worst <= tol) break;
                }
                if (t > T_max) t = T_max;
                plan_from_potentials(I, m, c, eps, f, g, X + (size_t)u * I * m);
                if (f_out) memcpy(f_out + (size_t)u * I, f, sizeof(double) * I);
                if (iters_out) iters_out[u] = t;
            }
        }
        free(f); free(gp); free(z);
    }
    return err;
}

/* Forward run to convergence: iterate until the largest row-marginal error of
 * the plan (columns are exact after every column half-step) is below tol, or
 * until cap iterations.  iters_out[u] receives the count used. */
ORC_EXPORT int fro_forward_converge(int64_t U, int I, int m, const double* C, double eps,
                                    double tol, int cap, double* X, double* f_out,
                                    double* g_out, int* iters_out) {
    if (check_shape(U, I, m) || !(eps > 0) || cap < 1 || !C || !X) return -1;
    int err = 0;
#pragma omp parallel
    {
        double* f = (double*)malloc(sizeof(double) * I);
        double* g = (double*)malloc(sizeof(double) * m);
        double* z = (double*)malloc(sizeof(double) * (I > m ? I : m));
        if (!f || !g || !z) {
#pragma omp atomic write
            err = -2;
        } else {
#pragma omp for schedule(static)
            for (int64_t u = 0; u < U; ++u) {
                const double* c = C + (size_t)u * I * m;
                double* Xu = X + (size_t)u * I * m;
                for (int k = 0; k < m; ++k) g[k] = 0.0;
                int t = 0;
                for (t = 1; t <= cap; ++t) {
                    sinkhorn_iter(I, m, c, eps, f, g, z);
                    plan_from_potentials(I, m, c, eps, f, g, Xu);
                    double worst = 0.0;
                    for (int i = 0; i < I; ++i) {
                        double s = 0.0;
                        for (int k = 0; k < m; ++k) s += Xu[(size_t)i * m + k];
                        if (fabs(s - 1.0) > worst) worst = fabs(s - 1.0);
                    }
                    if (worst < tol) break;
                }
                if (iters_out) iters_out[u] = t > cap ? cap : t;
                if (f_out) memcpy(f_out + (size_t)u * I, f, sizeof(double) * I);
                if (g_out) memcpy(g_out + (size_t)u * m, g, sizeof(double) * m);
            }
        }
        free(f); free(g); free(z);
    }
    return err;
}

/* Eq. Imp: Imp_i = sum_u sum_{k<m} r(u,i) e(k) x_uik; the dummy column has no
 * exposure.  Summed serially in consumer order. */
ORC_EXPORT int fro_impact(int64_t U, int I, int m, const double* r, const double* e,
                          const double* X, double* imp) {
    if (check_shape(U, I, m) || !r || !e || !X || !imp) return -1;
    for (int i = 0; i < I; ++i) imp[i] = 0.0;
    for (int64_t u = 0; u < U; ++u) {
        for (int i = 0; i < I; ++i) {
            double s = 0.0;
            for (int k = 0; k < m - 1; ++k) s += e[k] * X[((size_t)u * I + i) * m + k];
            imp[i] += r[(size_t)u * I + i] * s;
        }
    }
    return 0;
}

/* Eq. objF: F = sum_i log Imp_i. */
ORC_EXPORT double fro_nsw(int I, const double* imp) {
    double F = 0.0;
    for (int i = 0; i < I; ++i) F += log(imp[i]);
    return F;
}

/* Reverse mode through the T unrolled Sinkhorn iterations of one consumer.
 * Upstream gradient G_ik = dF/dx_ik = r_i e_k / Imp_i (k < m-1), 0 at the dummy.
 * fh [T][I] = f^1..f^T, gh [T+1][m] = g^0..g^T.  Writes gc [I][m]. */
static void reverse_one(int I, int m, const double* c, double eps, int T,
                        const double* ru, const double* e, const double* imp,
                        const double* fh, const double* gh, double* gc,
                        double* fbar, double* gbar, double* z, double* X, double* Mbuf) {
    const double* fT = fh + (size_t)(T - 1) * I;
    const double* gT = gh + (size_t)T * m;
    plan_from_potentials(I, m, c, eps, fT, gT, X);
    /* adjoints of X = exp((f + g - c)/eps) */
    for (int k = 0; k < m; ++k) gbar[k] = 0.0;
    for (int i = 0; i < I; ++i) {
        fbar[i] = 0.0;
        for (int k = 0; k < m; ++k) {
            double G = (k < m - 1) ? ru[i] * e[k] / imp[i] : 0.0;
            double gx = G * X[(size_t)i * m + k] / eps;
            gc[(size_t)i * m + k] = -gx;
            fbar[i] += gx;
            gbar[k] += gx;
        }
    }
    for (int t = T; t >= 1; --t) {
        const double* ft = fh + (size_t)(t - 1) * I;
        const double* gprev = gh + (size_t)(t - 1) * m;
        /* g^t_k = eps log b_k - eps LSE_i((f^t_i - c_ik)/eps):
         *   d g_k / d f_i = -Q_ik,  d g_k / d c_ik = +Q_ik,
         *   Q_ik = softmax over i of (f^t_i - c_ik)/eps.                  */
        for (int k = 0; k < m; ++k) {
            for (int i = 0; i < I; ++i) z[i] = (ft[i] - c[(size_t)i * m + k]) / eps;
            double l = lse(z, I, 1);
            for (int i = 0; i < I; ++i) {
                double Q = exp(z[i] - l);
                fbar[i] -= Q * gbar[k];
                gc[(size_t)i * m + k] += Q * gbar[k];
            }
        }
        /* f^t_i = -eps LSE_k((g^{t-1}_k - c_ik)/eps):
         *   d f_i / d g_k = -P_ik,  d f_i / d c_ik = +P_ik,
         *   P_ik = softmax over k of (g^{t-1}_k - c_ik)/eps.              */
        for (int k = 0; k < m; ++k) Mbuf[k] = 0.0;
        for (int i = 0; i < I; ++i) {
            for (int k = 0; k < m; ++k) z[k] = (gprev[k] - c[(size_t)i * m + k]) / eps;
            double l = lse(z, m, 1);
            for (int k = 0; k < m; ++k) {
                double P = exp(z[k] - l);
                Mbuf[k] -= P * fbar[i];
                gc[(size_t)i * m + k] += P * fbar[i];
            }
        }
        for (int k = 0; k < m; ++k) gbar[k] = Mbuf[k];
        /* f^{t-1} reaches f^t only through g^{t-1} */
        for (int i = 0; i < I; ++i) fbar[i] = 0.0;
    }
}

/* Gradient of F(X^(T)(C)) with respect to C and r, given the impacts of X(C).
 * gradC [U][I][m], gradr [U][I] (either may be NULL). */
ORC_EXPORT int fro_grad(int64_t U, int I, int m, const double* r, const double* e, double eps,
                        int T, const double* C, const double* imp, double* gradC,
                        double* gradr) {
    if (check_shape(U, I, m) || !(eps > 0) || T < 1 || !r || !e || !C || !imp) return -1;
    int err = 0;
#pragma omp parallel
    {
        double* f = (double*)malloc(sizeof(double) * I);
        double* g = (double*)malloc(sizeof(double) * m);
        double* z = (double*)malloc(sizeof(double) * (I > m ? I : m));
        double* fh = (double*)malloc(sizeof(double) * (size_t)T * I);
        double* gh = (double*)malloc(sizeof(double) * (size_t)(T + 1) * m);
        double* fbar = (double*)malloc(sizeof(double) * I);
        double* gbar = (double*)malloc(sizeof(double) * m);
        double* Mb = (double*)malloc(sizeof(double) * m);
        double* X = (double*)malloc(sizeof(double) * (size_t)I * m);
        double* gc = (double*)malloc(sizeof(double) * (size_t)I * m);
        if (!f || !g || !z || !fh || !gh || !fbar || !gbar || !Mb || !X || !gc) {
#pragma omp atomic write
            err = -2;
        } else {
#pragma omp for schedule(static)
            for (int64_t u = 0; u < U; ++u) {
                const double* c = C + (size_t)u * I * m;
                const double* ru = r + (size_t)u * I;
                sinkhorn_one(I, m, c, eps, T, f, g, z, fh, gh);
                reverse_one(I, m, c, eps, T, ru, e, imp, fh, gh, gc, fbar, gbar, z, X, Mb);
                if (gradC) memcpy(gradC + (size_t)u * I * m, gc, sizeof(double) * I * m);
                if (gradr) {
                    for (int i = 0; i < I; ++i) {
                        double s = 0.0;
                        for (int k = 0; k < m - 1; ++k) s += e[k] * X[(size_t)i * m + k];
                        gradr[(size_t)u * I + i] = s / imp[i];
                    }
                }
            }
        }
        free(f); free(g); free(z); free(fh); free(gh); free(fbar); free(gbar); free(Mb);
        free(X); free(gc);
    }
    return err;
}

/* Adam step for MAXIMISING F (Kingma & Ba, with bias correction as in
 * PyTorch's Adam, no weight decay): the minimised loss is -F, so its gradient
 * is -grad.  step is the 1-based step count t. */
ORC_EXPORT int fro_adam(int64_t n, double* C, double* mom, double* vel, const double* grad,
                        double lr, double b1, double b2, double aeps, int64_t step) {
    if (n < 0 || step < 1 || !C || !mom || !vel || !grad) return -1;
    double bc1 = 1.0 - pow(b1, (double)step);
    double bc2 = 1.0 - pow(b2, (double)step);
    for (int64_t j = 0; j < n; ++j) {
        double gl = -grad[j];
        mom[j] = b1 * mom[j] + (1.0 - b1) * gl;
        vel[j] = b2 * vel[j] + (1.0 - b2) * gl * gl;
        double mhat = mom[j] / bc1;
        double vhat = vel[j] / bc2;
        C[j] -= lr * mhat / (sqrt(vhat) + aeps);
    }
    return 0;
}

/* Plain gradient ascent: C <- C + lr * grad. */
ORC_EXPORT int fro_gd(int64_t n, double* C, const double* grad, double lr) {
    if (n < 0 || !C || !grad) return -1;
    for (int64_t j = 0; j < n; ++j) C[j] += lr * grad[j];
    return 0;
}

/* Algorithm 1 with at most N ascent steps:
 *   for n = 0..N: X = Sinkhorn_T(C); F_hist[n] = F(X); if n == N stop;
 *                 grad = dF/dC; if grad_tol > 0 and ||grad||_F <= grad_tol
 *                 stop (the loop condition of Algorithm 1); C <- update(C, grad).
 * After a stop C no longer changes, so F_hist[n+1..N] repeat F_hist[n].
 * rule 0 = Adam (mom, vel in/out; Adam step count start_step + updates + 1),
 * rule 1 = gradient ascent (mom, vel unused).
 * Outputs: C in place, X_out = X(C) (optional), F_hist [N+1], imp_out = Imp
 * (optional), gnorm_hist [N] = ||grad||_F of each step taken (optional),
 * updates_out = number of updates applied (optional). */
ORC_EXPORT int fro_solve(int64_t U, int I, int m, const double* r, const double* e, double eps,
                         int T, int N, int rule, double lr, double b1, double b2, double aeps,
                         double* C, double* mom, double* vel, int64_t start_step,
                         double* X_out, double* F_hist, double* imp_out, double grad_tol,
                         double* gnorm_hist, int64_t* updates_out) {
    if (check_shape(U, I, m) || !(eps > 0) || T < 1 || N < 0 || !r || !e || !C || !F_hist)
        return -1;
    if (rule == 0 && (!mom || !vel)) return -1;
    size_t n = (size_t)U * I * m;
    double* X = (double*)malloc(sizeof(double) * n);
    double* grad = (double*)malloc(sizeof(double) * n);
    double* imp = (double*)malloc(sizeof(double) * I);
    if (!X || !grad || !imp) { free(X); free(grad); free(imp); return -2; }
    int err = 0;
    int64_t updates = 0;
    int stopped = 0;
    for (int step = 0; step <= N; ++step) {
        if (stopped) {   /* the loop of Algorithm 1 has ended: C and F stay */
            F_hist[step] = F_hist[step - 1];
            continue;
        }
        if ((err = fro_forward(U, I, m, C, eps, T, X, NULL, NULL))) break;
        fro_impact(U, I, m, r, e, X, imp);
        F_hist[step] = fro_nsw(I, imp);
        if (step == N) break;
        if ((err = fro_grad(U, I, m, r, e, eps, T, C, imp, grad, NULL))) break;
        /* stopping test of Algorithm 1: ascend only while ||dF/dC||_F > t */
        double g2 = 0.0;
        for (size_t q = 0; q < n; ++q) g2 += grad[q] * grad[q];
        if (gnorm_hist) gnorm_hist[step] = sqrt(g2);
        if (grad_tol > 0.0 && sqrt(g2) <= grad_tol) {
            stopped = 1;
            continue;
        }
        if (rule == 0)
            fro_adam((int64_t)n, C, mom, vel, grad, lr, b1, b2, aeps, start_step + updates + 1);
        else
            fro_gd((int64_t)n, C, grad, lr);
        ++updates;
    }
    if (updates_out) *updates_out = updates;
    if (!err) {
        if (X_out) memcpy(X_out, X, sizeof(double) * n);
        if (imp_out) memcpy(imp_out, imp, sizeof(double) * I);
    }
    free(X); free(grad); free(imp);
    return err;
}

ORC_EXPORT int fro_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------------------
 * Baselines of the comparison in Section 4.1 (MaxRele, NSW(Greedy)).
 *
 * Both produce deterministic rankings: sel[u][k] is the item consumer u sees
 * at real position k (k < m-1, row-major [U][m-1]); every item not selected
 * by u goes to the dummy position.
 *
 * MaxRele: each consumer's items in descending order of relevance r(u,i);
 * equal relevances in increasing item index.
 *
 * NSW(Greedy): the paper says only that greedy picks items by F(X) for each
 * position.  Reading taken: the real positions are filled in order
 * k = 0 .. m-2; at each position the consumers choose in index order; a
 * consumer takes, among the items it has not placed yet, the one whose
 * placement at k raises F = sum_i log Imp_i (Eq. objF) the most.  Placing i
 * adds r(u,i) e(k) to Imp_i only, so the gain is
 *     log(Imp_i + r e_k) - log(Imp_i) = log(1 + e_k r / Imp_i),
 * increasing in r / Imp_i (e_k > 0 is the same for every candidate): the
 * choice is the largest ratio r(u,i) / Imp_i, an item with Imp_i = 0 counting
 * as +inf (its log goes from -inf to finite).  Equal ratios: larger r(u,i),
 * then smaller index.  Imp is accumulated in FP64 in decision order and
 * returned in imp[I].
 * ------------------------------------------------------------------------- */
ORC_EXPORT int fro_maxrele(int64_t U, int I, int m, const double* r, int32_t* sel) {
    if (U < 1 || I < 2 || m < 2 || m > I || !r || !sel) return -1;
    int* order = (int*)malloc(sizeof(int) * (size_t)I);
    if (!order) return -2;
    for (int64_t u = 0; u < U; ++u) {
        const double* ru = r + u * I;
        /* selection of the m-1 best, one position at a time */
        for (int i = 0; i < I; ++i) order[i] = 0;   /* 1 = already placed */
        for (int k = 0; k < m - 1; ++k) {
            int best = -1;
            for (int i = 0; i < I; ++i) {
                if (order[i]) continue;
                if (best < 0 || ru[i] > ru[best]) best = i;   /* ties keep the smaller index */
            }
            order[best] = 1;
            sel[u * (m - 1) + k] = best;
        }
    }
    free(order);
    return 0;
}

ORC_EXPORT int fro_greedy(int64_t U, int I, int m, const double* r, const double* e,
                          int32_t* sel, double* imp) {
    if (U < 1 || I < 2 || m < 2 || m > I || !r || !e || !sel || !imp) return -1;
    for (int i = 0; i < I; ++i) imp[i] = 0.0;
    for (int k = 0; k < m - 1; ++k) {
        for (int64_t u = 0; u < U; ++u) {
            const double* ru = r + u * I;
            const int32_t* mine = sel + u * (m - 1);
            int best = -1;
            double best_key = 0.0;
            for (int i = 0; i < I; ++i) {
                int placed = 0;
                for (int j = 0; j < k; ++j) placed |= (mine[j] == i);
                if (placed) continue;
                const double key = (imp[i] > 0.0) ? ru[i] / imp[i] : INFINITY;
                int better;
                if (best < 0) better = 1;
                else if (key != best_key) better = key > best_key;
                else better = ru[i] > ru[best];   /* then the smaller index stays */
                if (better) {
                    best = i;
                    best_key = key;
                }
            }
            sel[u * (m - 1) + k] = best;
            imp[best] += ru[best] * e[k];
        }
    }
    return 0;
}
