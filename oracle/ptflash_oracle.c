/*
 * ptflash_oracle.c -- plain, slow, scalar CPU oracle for the isothermal
 * two-phase PT flash with the Soave-Redlich-Kwong (SRK) equation of state,
 * following Qu, Faney, de Hemptinne, Yousef, Gallinari, "PTFlash: a deep
 * learning framework for isothermal two-phase equilibrium calculations"
 * (arXiv 2205.03090).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it; the library never does.  It
 * shares no code, header or constant table with the HIP path.
 *
 * Structure.  Where a step of the method reaches a result that has a plain
 * definition, this file computes that definition with a deliberately
 * different, plain method:
 *   - roots of the SRK cubic: all sign changes of the cubic in (B, 1+B),
 *     each bisected to adjacent doubles (the paper uses Halley + deflation);
 *   - the Rachford-Rice root: bisection to adjacent doubles on the window
 *     (1/(1-Kmax), 1/(1-Kmin)) (the paper uses Leibovici-Neoschil Newton);
 *   - stationary points of the modified tangent-plane distance and the
 *     converged phase split: damped Newton with a finite-difference Jacobian
 *     and Gaussian elimination with partial pivoting (the paper uses a
 *     trust-region method with analytic derivatives).
 * Where the method is a heuristic or an iteration whose path decides the
 * outcome (the Wilson start, the three initial successive substitutions and
 * their three-way triage, the two stability trials with their successive
 * substitution and iteration caps, the K re-estimate, the successive
 * substitution of the phase split with its cap), it follows the paper's
 * steps in the paper's order.
 *
 * Readings of passages that are silent, ambiguous or garbled:
 *   R1  modified tangent plane distance carries Michelsen's leading 1:
 *       tm(W) = 1 + sum W_i (ln W_i + ln phi_i(W) - d_i - 1)   (Sec. 2.2.1,
 *       eq. tm), so that tm = 0 at the trivial point W = z.
 *   R2  Delta G of the initial triage = (1-theta) tpd(x) + theta tpd(y)
 *       (Sec. 2.2.3); with theta in (0,1) it is a convex combination.
 *   R3  dominant-eigenvalue acceleration: at every 3rd successive
 *       substitution update u (u >= 2), lambda = (s_u . s_u)/(s_{u-1} . s_u)
 *       with s the plain update step; if 0 < lambda < 1 the update is
 *       extended by s_u lambda/(1-lambda).  The extrapolated point is kept
 *       only if its objective (tm for a stability trial, G per unit feed for
 *       the split) is lower than at the point the update started from, and,
 *       in the split, only if its Rachford-Rice root lies in (0,1) (where G
 *       is the Gibbs energy of two phases); otherwise the plain update is
 *       taken (the rejected evaluation is not counted).  A split update
 *       after which the substitution stops is never extended.  Not applied
 *       in the three initial iterations.  Period 3 is the one whose
 *       substitution convergence rates on the nine-component case study
 *       come closest to those of Table 5.
 *   R4  a stability trial is unstable when tm < -eps_tm (eps_tm = 1e-10).
 *   R5  trials start from the Wilson K; the initial successive substitution
 *       stops at the first iteration whose Rachford-Rice root leaves (0,1)
 *       (case 1); a case-3 split resumes from the latest K with a fresh
 *       budget of successive substitutions.
 *   R6  the root with the lowest Gibbs energy is chosen; a tie goes to the
 *       liquid (smaller) root.
 *   R7  compositions passed to the EOS are normalised to sum to one; after
 *       each Rachford-Rice solve x_i = z_i/(1+theta(K_i-1)), y_i = K_i x_i,
 *       both normalised.
 *   R8  the converged split is refined past the paper's 1e-8 criteria to
 *       the double-precision root of the equal-fugacity system.
 *   R9  canonical orientation of a two-phase result: y is the phase with
 *       the larger compressibility factor; single-phase results report
 *       x = y = z and beta = -1.
 *   R21 a split whose substitution leaves the two-phase region (no
 *       Rachford-Rice root, or theta outside (0,1)), or whose first descent
 *       ends at a degenerate split, at the trivial point x = y or
 *       unconverged with a phase below 1e-3 of the feed (stalled: kept, and
 *       the result, flagged unconverged, if the restarted descent ends
 *       degenerate or trivial), restarts once from n^V = beta w, w the
 *       composition that proved the instability (the stability trial the K
 *       re-estimate uses, or the triage's phase with the smaller tpd), beta
 *       halved from min(1, min z_i/w_i)/2 until G is below the feed's.
 *   R22 the K re-estimate never takes a trial whose tm is not a number.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define ORC_NCMAX 32

/* SRK constants as printed with the mixing and combining rules (Appendix A,
 * eqs. a_i and b_i), used unrounded-as-printed. */
#define ORC_OMEGA_A 0.42748
#define ORC_OMEGA_B 0.08664
/* Coefficient of the Wilson correlation (Sec. 2.2.1, eq. wilson). */
#define ORC_WILSON_C 5.373

/* ---------------------------------------------------------------------- */
/* Options and per-mixture record                                          */
/* ---------------------------------------------------------------------- */

typedef struct {
    int32_t max_pre_ss;      /* initial phase-split substitutions (3)      */
    int32_t max_ss;          /* successive-substitution cap (9)            */
    int32_t max_newton;      /* cap of the oracle's Newton stand-ins       */
    int32_t dem_every;       /* acceleration period (3), 0 = off           */
    int32_t want_min_tpd;    /* also compute the min-TPD diagnostic        */
    int32_t max_newton_split;/* cap of the split's Newton stand-in         */
    double tol_sa_ss;        /* max |d tm / d W| (1e-6)                    */
    double tol_sa_tr;        /* max |g| in beta variables (1e-6)           */
    double tol_split_ss;     /* max |K_new/K - 1| (1e-8)                   */
    double tol_split;        /* refinement target on the residual (1e-13)  */
    double eps_tm;           /* negative-tm threshold (1e-10)              */
    int32_t decision_only;   /* stop after the stability decision: label =
                                unstable, no phase split (0)               */
} orc_opts;

/* oracle-side outcome flags (independent of the library's status bits) */
#define ORC_INVALID        1u
#define ORC_SA_UNCONV      2u
#define ORC_SPLIT_UNCONV   4u
#define ORC_SPLIT_TRIVIAL  8u
#define ORC_SPLIT_FAILED  16u
#define ORC_RR_NO_ROOT    32u
#define ORC_HINTED        64u
#define ORC_SPLIT_RESTART 128u   /* split restarted from the unstable trial (R21) */

/* info[] layout per mixture */
enum {
    ORC_I_CASE = 0, ORC_I_PRE, ORC_I_SS_V, ORC_I_NT_V, ORC_I_SS_L, ORC_I_NT_L,
    ORC_I_SS_SPLIT, ORC_I_NT_SPLIT, ORC_I_FLAGS, ORC_I_OUT_V, ORC_I_OUT_L,
    ORC_I_NROOT_SWAP, ORC_I_SPLIT_SS_CONV, ORC_I_UNSTABLE, ORC_NINFO
};

/* ---------------------------------------------------------------------- */
/* EOS set-up: mixing and combining rules (Appendix A, eq. mixing_rule)    */
/* ---------------------------------------------------------------------- */

typedef struct {
    int nc;
    double Ai[ORC_NCMAX];                 /* a_i alpha_i P/(RT)^2         */
    double Bi[ORC_NCMAX];                 /* b_i P/(RT)                   */
    double Aij[ORC_NCMAX * ORC_NCMAX];    /* (a alpha)_ij P/(RT)^2        */
} orc_eos;

/* The gas constant cancels once a_i, b_i are scaled by P/(RT)^2 and P/(RT):
 * A_i = OMEGA_A alpha_i (Tc_i/T)^2 (P/Pc_i), B_i = OMEGA_B (Tc_i/T)(P/Pc_i). */
static void orc_eos_setup(int nc, const double *Tc, const double *Pc,
                          const double *omega, const double *kij,
                          double T, double P, orc_eos *e)
{
    e->nc = nc;
    for (int i = 0; i < nc; ++i) {
        double m = 0.480 + 1.574 * omega[i] - 0.176 * omega[i] * omega[i];
        double s = 1.0 + m * (1.0 - sqrt(T / Tc[i]));
        double alpha = s * s;
        double tr = Tc[i] / T;
        double pr = P / Pc[i];
        e->Ai[i] = ORC_OMEGA_A * alpha * tr * tr * pr;
        e->Bi[i] = ORC_OMEGA_B * tr * pr;
    }
    for (int i = 0; i < nc; ++i)
        for (int j = 0; j < nc; ++j)
            e->Aij[i * nc + j] = (1.0 - kij[i * nc + j]) * sqrt(e->Ai[i] * e->Ai[j]);
}

/* ---------------------------------------------------------------------- */
/* SRK cubic in Z (Appendix A, eq. cubic_Z) by bracketing bisection        */
/* ---------------------------------------------------------------------- */

static double orc_cubic_f(double Z, double r1, double r0)
{
    return ((Z - 1.0) * Z + r1) * Z - r0;
}

static double orc_bisect_cubic(double a, double b, double r1, double r0)
{
    double fa = orc_cubic_f(a, r1, r0), fb = orc_cubic_f(b, r1, r0);
    if (fa == 0.0) return a;
    if (fb == 0.0) return b;
    for (int it = 0; it < 4000; ++it) {
        double m = 0.5 * (a + b);
        if (!(m > a && m < b)) break;
        double fm = orc_cubic_f(m, r1, r0);
        if (fm == 0.0) return m;
        if ((fm < 0.0) == (fa < 0.0)) { a = m; fa = fm; }
        else { b = m; fb = fm; }
    }
    return fabs(fa) <= fabs(fb) ? a : b;
}

/* All real roots of Z^3 - Z^2 + (A - B - B^2) Z - AB in (B, 1+B), ascending.
 * The interval holds every root above B: f(B) = -2B^2 < 0, f(1+B) = A > 0
 * and f is increasing beyond 1+B.  It is split at the stationary points of f
 * so that each piece is monotonic, and each sign change is bisected. */
int orc_cubic_roots(double A, double B, double *roots)
{
    double r1 = A - B * (1.0 + B), r0 = A * B;
    double pts[4];
    int np = 0, nr = 0;
    pts[np++] = B;
    double disc = 1.0 - 3.0 * r1;
    if (disc > 0.0) {
        double s = sqrt(disc);
        double z1 = (1.0 - s) / 3.0, z2 = (1.0 + s) / 3.0;
        if (z1 > B && z1 < 1.0 + B) pts[np++] = z1;
        if (z2 > B && z2 < 1.0 + B) pts[np++] = z2;
    }
    pts[np++] = 1.0 + B;
    for (int k = 0; k + 1 < np; ++k) {
        double a = pts[k], b = pts[k + 1];
        double fa = orc_cubic_f(a, r1, r0), fb = orc_cubic_f(b, r1, r0);
        if (k > 0 && fa == 0.0) { roots[nr++] = a; continue; }
        if ((fa < 0.0 && fb > 0.0) || (fa > 0.0 && fb < 0.0))
            roots[nr++] = orc_bisect_cubic(a, b, r1, r0);
    }
    return nr;
}

/* Reduced residual Gibbs energy of one SRK root at fixed T, P and
 * composition; equals sum_i c_i ln phi_i (Appendix A, eq. lnphi). */
double orc_gres(double Z, double A, double B)
{
    return Z - 1.0 - log(Z - B) - (A / B) * log(1.0 + B / Z);
}

/* ---------------------------------------------------------------------- */
/* Fugacity coefficients of one phase (Appendix A, eq. lnphi)              */
/* ---------------------------------------------------------------------- */

typedef struct {
    double A, B, Z;
    int nroots;
    double roots[3];
} orc_phase_info;

static void orc_phase(const orc_eos *e, const double *c_in, double *lnphi,
                      orc_phase_info *info)
{
    int nc = e->nc;
    double c[ORC_NCMAX], psi[ORC_NCMAX], sum = 0.0;
    for (int i = 0; i < nc; ++i) sum += c_in[i];
    for (int i = 0; i < nc; ++i) c[i] = c_in[i] / sum;
    double A = 0.0, B = 0.0;
    for (int i = 0; i < nc; ++i) {
        double s = 0.0;
        for (int j = 0; j < nc; ++j) s += e->Aij[i * nc + j] * c[j];
        psi[i] = s;
    }
    for (int i = 0; i < nc; ++i) { A += c[i] * psi[i]; B += c[i] * e->Bi[i]; }
    double roots[3];
    int n = orc_cubic_roots(A, B, roots);
    double Z = roots[0];
    if (n > 1) {
        double zl = roots[0], zv = roots[n - 1];
        double gl = orc_gres(zl, A, B), gv = orc_gres(zv, A, B);
        Z = (gv < gl) ? zv : zl;          /* R6: tie goes to the liquid root */
    }
    double lzb = log(Z - B), l1 = log(1.0 + B / Z);
    for (int i = 0; i < nc; ++i) {
        double bb = e->Bi[i] / B;
        lnphi[i] = bb * (Z - 1.0) - lzb + (A / B) * (bb - 2.0 * psi[i] / A) * l1;
    }
    if (info) {
        info->A = A; info->B = B; info->Z = Z; info->nroots = n;
        for (int k = 0; k < 3; ++k) info->roots[k] = k < n ? roots[k] : 0.0;
    }
}

/* ---------------------------------------------------------------------- */
/* Wilson K (Sec. 2.2.1, eq. wilson)                                       */
/* ---------------------------------------------------------------------- */

static void orc_wilson(int nc, const double *Tc, const double *Pc,
                       const double *omega, double T, double P, double *lnK)
{
    for (int i = 0; i < nc; ++i)
        lnK[i] = log(Pc[i] / P) + ORC_WILSON_C * (1.0 + omega[i]) * (1.0 - Tc[i] / T);
}

/* ---------------------------------------------------------------------- */
/* Rachford-Rice (Sec. 2.2.2, eq. RR; Appendix C) by bisection             */
/* ---------------------------------------------------------------------- */

static double orc_rr_f(int nc, const double *z, const double *K, double th)
{
    double f = 0.0;
    for (int i = 0; i < nc; ++i) f += (K[i] - 1.0) * z[i] / (1.0 + (K[i] - 1.0) * th);
    return f;
}

/* Root of f_RR in the window (1/(1-Kmax), 1/(1-Kmin)) where every phase
 * composition stays positive; f_RR decreases from +inf to -inf across it.
 * Returns 0 with *theta, -1 when all K <= 1, +1 when all K >= 1. */
int orc_rr_solve(int nc, const double *z, const double *K, double *theta)
{
    double kmax = K[0], kmin = K[0];
    for (int i = 1; i < nc; ++i) {
        if (K[i] > kmax) kmax = K[i];
        if (K[i] < kmin) kmin = K[i];
    }
    if (kmax <= 1.0) return -1;
    if (kmin >= 1.0) return 1;
    double a = 1.0 / (1.0 - kmax), b = 1.0 / (1.0 - kmin);
    double fa = INFINITY, fb = -INFINITY;
    for (int it = 0; it < 4000; ++it) {
        double m = 0.5 * (a + b);
        if (!(m > a && m < b)) break;
        double fm = orc_rr_f(nc, z, K, m);
        if (fm == 0.0) { *theta = m; return 0; }
        if (fm > 0.0) { a = m; fa = fm; } else { b = m; fb = fm; }
    }
    *theta = fabs(fa) <= fabs(fb) ? a : b;
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Small dense linear algebra: Gaussian elimination, partial pivoting      */
/* ---------------------------------------------------------------------- */

/* Solves M x = rhs in place (M is n x n row-major, destroyed).  Returns 0 on
 * success, 1 when a pivot vanishes. */
static int orc_gepp(int n, double *M, double *rhs)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(M[k * n + k]);
        for (int r = k + 1; r < n; ++r)
            if (fabs(M[r * n + k]) > best) { best = fabs(M[r * n + k]); p = r; }
        if (!(best > 0.0) || !isfinite(best)) return 1;
        if (p != k) {
            for (int c = 0; c < n; ++c) {
                double t = M[k * n + c]; M[k * n + c] = M[p * n + c]; M[p * n + c] = t;
            }
            double t = rhs[k]; rhs[k] = rhs[p]; rhs[p] = t;
        }
        for (int r = k + 1; r < n; ++r) {
            double f = M[r * n + k] / M[k * n + k];
            for (int c = k; c < n; ++c) M[r * n + c] -= f * M[k * n + c];
            rhs[r] -= f * rhs[k];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        double s = rhs[k];
        for (int c = k + 1; c < n; ++c) s -= M[k * n + c] * rhs[c];
        rhs[k] = s / M[k * n + k];
    }
    return 0;
}

/* 1 when the symmetric n x n matrix M is positive definite: Gaussian
 * elimination without pivoting (the LDL^T factorisation) has only positive
 * pivots (Sylvester's criterion).  M is not modified. */
static int orc_pos_def(int n, const double *M)
{
    double A[ORC_NCMAX * ORC_NCMAX];
    memcpy(A, M, sizeof(double) * n * n);
    for (int k = 0; k < n; ++k) {
        if (!(A[k * n + k] > 0.0) || !isfinite(A[k * n + k])) return 0;
        for (int r = k + 1; r < n; ++r) {
            double f = A[r * n + k] / A[k * n + k];
            for (int c = k; c < n; ++c) A[r * n + c] -= f * A[k * n + c];
        }
    }
    return 1;
}

/* ---------------------------------------------------------------------- */
/* Tangent plane distances (Sec. 2.2.1, eqs. tpd and tm)                   */
/* ---------------------------------------------------------------------- */

/* tpd(w) = sum w_i (ln w_i + ln phi_i(w) - d_i), d_i = ln z_i + ln phi_i(z) */
static double orc_tpd(const orc_eos *e, const double *w_in, const double *d)
{
    int nc = e->nc;
    double w[ORC_NCMAX], lp[ORC_NCMAX], s = 0.0, t = 0.0;
    for (int i = 0; i < nc; ++i) s += w_in[i];
    for (int i = 0; i < nc; ++i) w[i] = w_in[i] / s;
    orc_phase(e, w, lp, NULL);
    for (int i = 0; i < nc; ++i) t += w[i] * (log(w[i]) + lp[i] - d[i]);
    return t;
}

/* Stability-trial state at mole numbers W = exp(lnW): gradient of tm with
 * respect to W (ln W + ln phi(W) - d), and tm with the leading 1 (R1). */
static double orc_tm_eval(const orc_eos *e, const double *lnW, const double *d,
                          double *grad, double *lnphi_out)
{
    int nc = e->nc;
    double W[ORC_NCMAX], lp[ORC_NCMAX];
    for (int i = 0; i < nc; ++i) W[i] = exp(lnW[i]);
    orc_phase(e, W, lp, NULL);
    double tm = 1.0;
    for (int i = 0; i < nc; ++i) {
        grad[i] = lnW[i] + lp[i] - d[i];
        tm += W[i] * (grad[i] - 1.0);
        if (lnphi_out) lnphi_out[i] = lp[i];
    }
    return tm;
}

enum { ORC_TRIAL_STATIONARY = 0, ORC_TRIAL_NEGATIVE = 1, ORC_TRIAL_UNCONV = 2 };

/* Successive substitution of a stability trial (Sec. 2.2.1, eq.
 * ss_analyser), ln W <- d - ln phi(W), accelerated per R3.  Each iteration
 * first evaluates the stopping tests at the current W: tm < -eps (unstable)
 * or max |d tm/d W| < tol (stationary).  After max_ss updates without a stop
 * the caller continues with a second-order method. */
static int orc_sa_ss(const orc_eos *e, const double *d, double *lnW,
                     const orc_opts *o, int *n_upd, double *tm_out)
{
    int nc = e->nc;
    double grad[ORC_NCMAX], step[ORC_NCMAX], prev[ORC_NCMAX];
    int upd = 0, pending = 0;
    double tm_before = 0.0, ext_applied = 0.0;
    *n_upd = 0;
    for (int guard = 0; guard < 4 * o->max_ss + 8; ++guard) {
        double tm = orc_tm_eval(e, lnW, d, grad, NULL);
        *tm_out = tm;
        if (tm < -o->eps_tm) return ORC_TRIAL_NEGATIVE;
        double gmax = 0.0;
        for (int i = 0; i < nc; ++i) if (fabs(grad[i]) > gmax) gmax = fabs(grad[i]);
        if (gmax < o->tol_sa_ss) return ORC_TRIAL_STATIONARY;
        if (pending) {
            /* R3: an extrapolated point is kept only if it lowers tm */
            pending = 0;
            if (!(tm < tm_before)) {
                for (int i = 0; i < nc; ++i) lnW[i] -= ext_applied * prev[i];
                continue;
            }
        }
        if (upd == o->max_ss) return ORC_TRIAL_UNCONV;
        for (int i = 0; i < nc; ++i) step[i] = -grad[i];
        ++upd;
        double ext = 0.0;
        if (o->dem_every > 0 && upd >= 2 && upd % o->dem_every == 0) {
            double num = 0.0, den = 0.0;
            for (int i = 0; i < nc; ++i) { num += step[i] * step[i]; den += prev[i] * step[i]; }
            double lam = num / den;
            if (lam > 0.0 && lam < 1.0) ext = lam / (1.0 - lam);
        }
        for (int i = 0; i < nc; ++i) {
            lnW[i] += step[i] + ext * step[i];
            prev[i] = step[i];
        }
        if (ext > 0.0) { pending = 1; tm_before = tm; ext_applied = ext; }
        *n_upd = upd;
    }
    return ORC_TRIAL_UNCONV;
}

/* Gradient of tm with respect to beta = 2 sqrt(W) (Appendix B.1, eq.
 * analysis_grad): g_i = sqrt(W_i) (ln W_i + ln phi_i - d_i). */
static double orc_sa_gbeta(const orc_eos *e, const double *d, const double *beta,
                           double *g)
{
    int nc = e->nc;
    double lnW[ORC_NCMAX], grad[ORC_NCMAX];
    for (int i = 0; i < nc; ++i) lnW[i] = 2.0 * log(0.5 * beta[i]);
    double tm = orc_tm_eval(e, lnW, d, grad, NULL);
    for (int i = 0; i < nc; ++i) g[i] = 0.5 * beta[i] * grad[i];
    return tm;
}

/* ---------------------------------------------------------------------- */
/* Damped Newton minimiser (oracle's stand-in for the trust regions)       */
/* ---------------------------------------------------------------------- */

/* Objective callback: returns the value at x and writes the gradient. */
typedef double (*orc_objfn)(void *ctx, const double *x, double *grad);
/* Diagonal metric callback: writes positive scaling entries at x. */
typedef void (*orc_metricfn)(void *ctx, const double *x, double *dm);

typedef struct {
    int n;
    orc_objfn fn;
    orc_metricfn metric;
    void *ctx;
    const double *lo, *hi;   /* open box lo < x < hi (hi may be NULL)      */
    double fd_rel;           /* relative finite-difference step            */
    double tol;              /* stop at max |grad| < tol                   */
    double stop_below;       /* stop when f < stop_below (-INF: never)     */
    int max_it;
} orc_minprob;

enum { ORC_MIN_TOL = 0, ORC_MIN_BELOW = 1, ORC_MIN_CAP = 2, ORC_MIN_STUCK = 3 };

/* Newton's method on grad f = 0 with a symmetric central-difference Hessian,
 * Levenberg-Marquardt damping (H + mu D) p = -grad in the metric D whenever
 * H is not positive definite or the line search cuts the step,
 * a fraction-to-the-boundary rule for the box, and Armijo backtracking on f.
 * Close to the stationary point (max |grad| < 1e-5), where f may change
 * less than its rounding, a step that fails Armijo is still accepted when it
 * lowers the gradient and does not raise f beyond rounding (1e-13 |f|): the
 * method stays a descent method, like the paper's trust regions, whose steps
 * are judged on the decrease of the objective (Appendix B). */
static int orc_minimise(const orc_minprob *pr, double *x, int *n_it, double *f_out)
{
    int n = pr->n;
    double g[ORC_NCMAX], gp[ORC_NCMAX], gm[ORC_NCMAX], H[ORC_NCMAX * ORC_NCMAX];
    double M[ORC_NCMAX * ORC_NCMAX], p[ORC_NCMAX], xt[ORC_NCMAX], gt[ORC_NCMAX];
    double dm[ORC_NCMAX];
    double mu = 0.0, best = INFINITY;
    int stall = 0;
    *n_it = 0;
    for (int it = 0;; ++it) {
        double f = pr->fn(pr->ctx, x, g);
        *f_out = f;
        if (f < pr->stop_below) return ORC_MIN_BELOW;
        double gmax = 0.0;
        for (int i = 0; i < n; ++i) if (fabs(g[i]) > gmax) gmax = fabs(g[i]);
        if (!(gmax == gmax)) return ORC_MIN_STUCK;
        if (gmax < pr->tol) return ORC_MIN_TOL;
        int local = gmax < 1e-5;
        if (local) {
            if (gmax < best) { best = gmax; stall = 0; }
            else if (++stall >= 3) return ORC_MIN_STUCK;
            mu = 0.0;   /* plain Newton first near the stationary point */
        }
        if (it == pr->max_it) return ORC_MIN_CAP;
        *n_it = it + 1;
        for (int j = 0; j < n; ++j) {
            double span = x[j] - pr->lo[j];
            if (pr->hi && pr->hi[j] - x[j] < span) span = pr->hi[j] - x[j];
            double h = pr->fd_rel * span;
            memcpy(xt, x, sizeof(double) * n);
            xt[j] = x[j] + h; pr->fn(pr->ctx, xt, gp);
            xt[j] = x[j] - h; pr->fn(pr->ctx, xt, gm);
            for (int i = 0; i < n; ++i) H[i * n + j] = (gp[i] - gm[i]) / (2.0 * h);
        }
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < i; ++j) {
                double a = 0.5 * (H[i * n + j] + H[j * n + i]);
                H[i * n + j] = a; H[j * n + i] = a;
            }
        pr->metric(pr->ctx, x, dm);
        double hscale = 0.0;
        for (int i = 0; i < n; ++i) hscale = fmax(hscale, fabs(H[i * n + i]) / dm[i]);
        if (!(hscale > 0.0)) hscale = 1.0;
        double slope = 0.0;
        int tries = 0;
        for (;; ++tries) {
            memcpy(M, H, sizeof(double) * n * n);
            for (int i = 0; i < n; ++i) { M[i * n + i] += mu * dm[i]; p[i] = -g[i]; }
            /* the model must be convex (as a trust-region step's shifted
             * Hessian is): with an indefinite H the Newton step heads for a
             * saddle, such as the trivial point of an unstable feed */
            int bad = !orc_pos_def(n, M) || orc_gepp(n, M, p);
            slope = 0.0;
            for (int i = 0; i < n; ++i) slope += g[i] * p[i];
            if (!bad && slope < 0.0) break;
            if (tries > 60) return ORC_MIN_STUCK;
            mu = mu > 0.0 ? 10.0 * mu : 1e-6 * hscale;
        }
        double amax = 1.0;
        for (int i = 0; i < n; ++i) {
            if (p[i] < 0.0) amax = fmin(amax, 0.99 * (x[i] - pr->lo[i]) / -p[i]);
            if (pr->hi && p[i] > 0.0) amax = fmin(amax, 0.99 * (pr->hi[i] - x[i]) / p[i]);
        }
        double a = amax;
        int acc = 0, cuts = 0;
        for (; cuts < 60; ++cuts) {
            for (int i = 0; i < n; ++i) xt[i] = x[i] + a * p[i];
            double ft = pr->fn(pr->ctx, xt, gt);
            /* sufficient decrease of the objective (Armijo) ... */
            acc = ft <= f + 1e-4 * a * slope;
            if (!acc && local) {
                /* ... or, near a stationary point where the decrease is at
                 * the rounding level of f, a smaller gradient with f not
                 * above rounding of its current value (a descent method:
                 * it never climbs to a saddle such as the trivial point) */
                double tmax = 0.0, t2 = 0.0, g2 = 0.0;
                for (int i = 0; i < n; ++i) {
                    if (fabs(gt[i]) > tmax) tmax = fabs(gt[i]);
                    t2 += gt[i] * gt[i];
                    g2 += g[i] * g[i];
                }
                acc = (tmax < gmax || t2 < g2) && ft <= f + 1e-13 * fmax(1.0, fabs(f));
            }
            if (acc) break;
            a *= 0.5;
        }
        if (!acc) {
            if (mu > 1e12 * hscale) return ORC_MIN_STUCK;
            mu = mu > 0.0 ? 10.0 * mu : 1e-6 * hscale;
            continue;
        }
        memcpy(x, xt, sizeof(double) * n);
        if (cuts == 0) mu *= 0.1;
        else if (cuts > 3) mu = mu > 0.0 ? 10.0 * mu : 1e-6 * hscale;
        if (mu < 1e-12 * hscale) mu = 0.0;
    }
}

/* tm and its gradient over beta = 2 sqrt(W) (Appendix B.1). */
typedef struct { const orc_eos *e; const double *d; } orc_sa_ctx;

static double orc_sa_obj(void *ctx, const double *beta, double *g)
{
    orc_sa_ctx *c = (orc_sa_ctx *)ctx;
    return orc_sa_gbeta(c->e, c->d, beta, g);
}

static void orc_unit_metric(void *ctx, const double *x, double *dm)
{
    orc_sa_ctx *c = (orc_sa_ctx *)ctx;
    (void)x;
    for (int i = 0; i < c->e->nc; ++i) dm[i] = 1.0;
}

/* Stand-in for the stability trust region (Appendix B.1): a stationary
 * point of tm over beta = 2 sqrt(W) by the damped Newton minimiser above.
 * Stops on tm < -eps (when stop_negative) or max |g| < tol. */
static int orc_sa_newton(const orc_eos *e, const double *d, double *lnW,
                         const orc_opts *o, double tol, int stop_negative,
                         int *n_it, double *tm_out)
{
    int nc = e->nc;
    double beta[ORC_NCMAX], lo[ORC_NCMAX];
    for (int i = 0; i < nc; ++i) { beta[i] = 2.0 * exp(0.5 * lnW[i]); lo[i] = 0.0; }
    orc_sa_ctx c = {e, d};
    orc_minprob pr = {nc, orc_sa_obj, orc_unit_metric, &c, lo, NULL, 1e-6, tol,
                      stop_negative ? -o->eps_tm : -INFINITY, o->max_newton};
    int rc = orc_minimise(&pr, beta, n_it, tm_out);
    for (int i = 0; i < nc; ++i) lnW[i] = 2.0 * log(0.5 * beta[i]);
    if (rc == ORC_MIN_BELOW) return ORC_TRIAL_NEGATIVE;
    if (rc == ORC_MIN_TOL) return ORC_TRIAL_STATIONARY;
    if (rc == ORC_MIN_STUCK && tol < 1e-9) {
        /* at the rounding floor of a tight diagnostic tolerance */
        double g[ORC_NCMAX], gmax = 0.0;
        orc_sa_gbeta(e, d, beta, g);
        for (int i = 0; i < nc; ++i) gmax = fmax(gmax, fabs(g[i]));
        if (gmax < 1e-9) return ORC_TRIAL_STATIONARY;
    }
    return ORC_TRIAL_UNCONV;
}

/* ---------------------------------------------------------------------- */
/* Phase split (Sec. 2.2.2; Appendix B.2)                                  */
/* ---------------------------------------------------------------------- */

/* x, y from K through the Rachford-Rice root (R7). */
static void orc_xy_from_k(int nc, const double *z, const double *K, double th,
                          double *x, double *y)
{
    double sx = 0.0, sy = 0.0;
    for (int i = 0; i < nc; ++i) {
        x[i] = z[i] / (1.0 + th * (K[i] - 1.0));
        y[i] = K[i] * x[i];
        sx += x[i]; sy += y[i];
    }
    for (int i = 0; i < nc; ++i) { x[i] /= sx; y[i] /= sy; }
}

/* Residual of the equal-fugacity system in the vapour mole numbers nV
 * (Appendix B.2, eq. split_grad): r_i = ln y_i + ln phi_i(y) - ln x_i -
 * ln phi_i(x), with x = (z - nV)/(1 - sum nV), y = nV / sum nV.  Also
 * returns the reduced Gibbs energy G of eq. gibbs (through *G). */
static void orc_split_res(const orc_eos *e, const double *z, const double *nV,
                          double *r, double *G)
{
    int nc = e->nc;
    double x[ORC_NCMAX], y[ORC_NCMAX], lx[ORC_NCMAX], ly[ORC_NCMAX];
    double bv = 0.0;
    for (int i = 0; i < nc; ++i) bv += nV[i];
    for (int i = 0; i < nc; ++i) { y[i] = nV[i] / bv; x[i] = (z[i] - nV[i]) / (1.0 - bv); }
    orc_phase(e, x, lx, NULL);
    orc_phase(e, y, ly, NULL);
    double g = 0.0;
    for (int i = 0; i < nc; ++i) {
        double fx = log(x[i]) + lx[i], fy = log(y[i]) + ly[i];
        r[i] = fy - fx;
        g += (z[i] - nV[i]) * fx + nV[i] * fy;
    }
    if (G) *G = g;
}

/* Successive substitution of the phase split (Sec. 2.2.2): RR -> x, y ->
 * ln K <- ln phi(x) - ln phi(y); stops at max |K_new/K - 1| < tol or after
 * max_ss updates; accelerated per R3.  Returns the number of updates, sets
 * *conv, and leaves ln K at the last update. */
static int orc_split_ss(const orc_eos *e, const double *z, double *lnK,
                        const orc_opts *o, int *conv, int *rr_fail)
{
    int nc = e->nc;
    double K[ORC_NCMAX], x[ORC_NCMAX], y[ORC_NCMAX], lx[ORC_NCMAX], ly[ORC_NCMAX];
    double step[ORC_NCMAX], prev[ORC_NCMAX];
    int u = 0, pending = 0;
    double g_before = 0.0, ext_applied = 0.0;
    *conv = 0; *rr_fail = 0;
    for (int guard = 0; guard < 4 * o->max_ss + 8 && u < o->max_ss; ++guard) {
        double th;
        for (int i = 0; i < nc; ++i) K[i] = exp(lnK[i]);
        if (orc_rr_solve(nc, z, K, &th) != 0) {
            if (pending) {
                /* R3: an extrapolated point without a Rachford-Rice root is
                 * rejected like one that does not lower G */
                pending = 0;
                for (int i = 0; i < nc; ++i) lnK[i] -= ext_applied * prev[i];
                continue;
            }
            *rr_fail = 1;
            return u;
        }
        orc_xy_from_k(nc, z, K, th, x, y);
        orc_phase(e, x, lx, NULL);
        orc_phase(e, y, ly, NULL);
        /* reduced Gibbs energy per unit feed at this point (eq. gibbs) */
        double G = 0.0;
        if (pending || (o->dem_every > 0 && (u + 1) >= 2 && (u + 1) % o->dem_every == 0)) {
            for (int i = 0; i < nc; ++i)
                G += (1.0 - th) * x[i] * (log(x[i]) + lx[i]) + th * y[i] * (log(y[i]) + ly[i]);
        }
        if (pending) {
            /* R3: an extrapolated point is kept only if it is a physical
             * split (0 < theta < 1, where eq. gibbs is the Gibbs energy of
             * two phases) and lowers G */
            pending = 0;
            if (!(th > 0.0 && th < 1.0 && G < g_before)) {
                for (int i = 0; i < nc; ++i) lnK[i] -= ext_applied * prev[i];
                continue;
            }
        }
        double dmax = 0.0;
        for (int i = 0; i < nc; ++i) {
            step[i] = (lx[i] - ly[i]) - lnK[i];
            double q = fabs(exp(step[i]) - 1.0);
            if (q > dmax) dmax = q;
        }
        ++u;
        /* R3: no extension on an update after which the substitution stops
         * (converged or out of budget), since no later evaluation could
         * check the extrapolated point */
        int more = !(dmax < o->tol_split_ss) && u < o->max_ss;
        double ext = 0.0;
        if (more && o->dem_every > 0 && u >= 2 && u % o->dem_every == 0) {
            double num = 0.0, den = 0.0;
            for (int i = 0; i < nc; ++i) { num += step[i] * step[i]; den += prev[i] * step[i]; }
            double lam = num / den;
            if (lam > 0.0 && lam < 1.0) ext = lam / (1.0 - lam);
        }
        for (int i = 0; i < nc; ++i) { lnK[i] += step[i] + ext * step[i]; prev[i] = step[i]; }
        if (dmax < o->tol_split_ss) { *conv = 1; return u; }
        if (ext > 0.0) { pending = 1; g_before = G; ext_applied = ext; }
    }
    return u;
}

/* R21: start of the phase split from a composition w with negative
 * tangent-plane distance, when the substitution left the two-phase region:
 * n^V = beta w with beta = min(1, min_i z_i / w_i) / 2, halved (at most 30
 * times) until the split's G per unit feed is below the feed's, G_feed =
 * sum z_i d_i, by more than 1e-12 (1 + |G_feed|).  For small beta,
 * G - G_feed = beta tpd(w) + O(beta^2) < 0.  Returns 0 and n^V on success. */
static int orc_split_restart(const orc_eos *e, const double *z, const double *d,
                             const double *w, double *nV)
{
    int nc = e->nc;
    double gf = 0.0, bmax = 1.0, r[ORC_NCMAX];
    for (int i = 0; i < nc; ++i) {
        gf += z[i] * d[i];
        if (z[i] / w[i] < bmax) bmax = z[i] / w[i];
    }
    double beta = 0.5 * bmax;
    for (int h = 0; h <= 30; ++h, beta *= 0.5) {
        for (int i = 0; i < nc; ++i) nV[i] = beta * w[i];
        double G;
        orc_split_res(e, z, nV, r, &G);
        if (G < gf - 1e-12 * (1.0 + fabs(gf))) return 0;
    }
    return 1;
}

/* G and its gradient over the vapour mole numbers (eqs. gibbs, split_grad). */
typedef struct { const orc_eos *e; const double *z; } orc_split_ctx;

static double orc_split_obj(void *ctx, const double *nV, double *r)
{
    orc_split_ctx *c = (orc_split_ctx *)ctx;
    double G;
    orc_split_res(c->e, c->z, nV, r, &G);
    return G;
}

/* Ideal-mixing part of the Hessian of G: z_i / (nV_i (z_i - nV_i)). */
static void orc_split_metric(void *ctx, const double *nV, double *dm)
{
    orc_split_ctx *c = (orc_split_ctx *)ctx;
    for (int i = 0; i < c->e->nc; ++i) dm[i] = c->z[i] / (nV[i] * (c->z[i] - nV[i]));
}

/* Stand-in for the phase-split trust region (Appendix B.2) and the
 * refinement R8: the damped Newton minimiser on G over 0 < nV < z, run to
 * max |r| < tol (or to the rounding floor, accepted below 1e-9). */
static int orc_split_newton(const orc_eos *e, const double *z, double *nV,
                            const orc_opts *o, int *n_it)
{
    int nc = e->nc;
    double lo[ORC_NCMAX], G, r[ORC_NCMAX];
    for (int i = 0; i < nc; ++i) lo[i] = 0.0;
    orc_split_ctx c = {e, z};
    orc_minprob pr = {nc, orc_split_obj, orc_split_metric, &c, lo, z, 1e-7,
                      o->tol_split, -INFINITY, o->max_newton_split};
    int rc = orc_minimise(&pr, nV, n_it, &G);
    if (rc == ORC_MIN_TOL) return 0;
    if (rc == ORC_MIN_STUCK) {
        double rmax = 0.0;
        orc_split_res(e, z, nV, r, NULL);
        for (int i = 0; i < nc; ++i) rmax = fmax(rmax, fabs(r[i]));
        if (rmax < 1e-9) return 0;
    }
    return 1;
}

/* ---------------------------------------------------------------------- */
/* The flash (Sec. 2.2.3 strategy; Algorithm 2 for stability analysis)     */
/* ---------------------------------------------------------------------- */

typedef struct {
    int label;
    double beta, min_tpd;
    double tm_dec;   /* the value that decided stability (see orc_flash_one) */
    double x[ORC_NCMAX], y[ORC_NCMAX];
    int32_t info[ORC_NINFO];
} orc_result;

static int orc_is_trivial(int nc, const double *lnW, const double *z)
{
    double m = 0.0, s = 0.0;
    for (int i = 0; i < nc; ++i) s += exp(lnW[i]);
    for (int i = 0; i < nc; ++i) { double q = fabs(lnW[i] - log(s) - log(z[i])); if (q > m) m = q; }
    return m < 1e-4;
}

/* A split n^V of the feed z whose phases coincide: max_i |ln(y_i/x_i)| below
 * 1e-6 (the test the result uses to report a trivial split). */
static int orc_split_is_trivial(int nc, const double *z, const double *nV, double bv)
{
    if (!(bv > 1e-10 && bv < 1.0 - 1e-10)) return 0;
    double bl = 0.0, lkmax = 0.0;
    for (int i = 0; i < nc; ++i) bl += z[i] - nV[i];
    for (int i = 0; i < nc; ++i) {
        double q = fabs(log((nV[i] / bv) / ((z[i] - nV[i]) / bl)));
        if (q > lkmax) lkmax = q;
    }
    return lkmax < 1e-6;
}

static void orc_single_phase(int nc, const double *z, orc_result *res)
{
    res->label = 0;
    res->beta = -1.0;
    for (int i = 0; i < nc; ++i) { res->x[i] = z[i]; res->y[i] = z[i]; }
}

/* lnk0 (nullable): the caller's initial ln K in place of Wilson's, wherever
 * the flash uses Wilson's (the first substitutions, the two stability trials
 * and the split of a hinted-unstable mixture; Sec. 4).  hint: 0 = known stable (single phase, no analysis), 1 =
 * known unstable (the split starts from the initial K without the triage and
 * the stability analysis; case 4 in info), other values: none. */
int orc_flash_one(int nc, const double *z_in, double T, double P,
                  const double *Tc, const double *Pc, const double *omega,
                  const double *kij, const double *lnk0, int hint, const orc_opts *o,
                  orc_result *res)
{
    memset(res, 0, sizeof(*res));
    res->min_tpd = NAN;
    res->tm_dec = NAN;
    orc_single_phase(nc, z_in, res);
    res->info[ORC_I_FLAGS] = ORC_INVALID;
    if (nc < 1 || nc > ORC_NCMAX || !(T > 0.0) || !(P > 0.0) || !isfinite(T) || !isfinite(P))
        return ORC_INVALID;
    double zs = 0.0;
    for (int i = 0; i < nc; ++i) {
        if (!(z_in[i] > 0.0) || !isfinite(z_in[i]) || !(Tc[i] > 0.0) || !(Pc[i] > 0.0) ||
            !isfinite(omega[i]))
            return ORC_INVALID;
        zs += z_in[i];
        for (int j = 0; j < nc; ++j)
            if (kij[i * nc + j] != kij[j * nc + i] || (i == j && kij[i * nc + i] != 0.0))
                return ORC_INVALID;
        if (lnk0 && !isfinite(lnk0[i])) return ORC_INVALID;
    }
    res->info[ORC_I_FLAGS] = 0;
    unsigned flags = 0;
    if (hint == 0) {
        double zn[ORC_NCMAX];
        for (int i = 0; i < nc; ++i) zn[i] = z_in[i] / zs;
        orc_single_phase(nc, zn, res);
        res->info[ORC_I_FLAGS] = ORC_HINTED;
        return 0;
    }

    double z[ORC_NCMAX], lnz[ORC_NCMAX];
    for (int i = 0; i < nc; ++i) { z[i] = z_in[i] / zs; lnz[i] = log(z[i]); }
    orc_single_phase(nc, z, res);

    orc_eos e;
    orc_eos_setup(nc, Tc, Pc, omega, kij, T, P, &e);

    /* feed reference d_i = ln z_i + ln phi_i(z) (eq. tpd) */
    double d[ORC_NCMAX], lpz[ORC_NCMAX];
    orc_phase(&e, z, lpz, NULL);
    for (int i = 0; i < nc; ++i) d[i] = lnz[i] + lpz[i];

    double lnKw[ORC_NCMAX], lnK[ORC_NCMAX], K[ORC_NCMAX];
    if (lnk0) memcpy(lnKw, lnk0, sizeof(double) * nc);
    else orc_wilson(nc, Tc, Pc, omega, T, P, lnKw);
    memcpy(lnK, lnKw, sizeof(double) * nc);

    /* Three initial substitutions of the phase split and the triage (Sec.
     * 2.2.3): case 1 = theta left (0,1); case 3 = some of tpd(x), tpd(y),
     * Delta G negative (unstable, no stability analysis); case 2 otherwise. */
    int kase = 0, npre = 0;
    double th = 0.0, x[ORC_NCMAX], y[ORC_NCMAX], lx[ORC_NCMAX], ly[ORC_NCMAX];
    double tpdx = INFINITY, tpdy = INFINITY;
    if (hint == 1) {
        kase = 4;   /* the caller's hint: unstable, no triage */
        flags |= ORC_HINTED;
    }
    for (int k = 1; kase != 4 && k <= o->max_pre_ss; ++k) {
        for (int i = 0; i < nc; ++i) K[i] = exp(lnK[i]);
        if (orc_rr_solve(nc, z, K, &th) != 0 || !(th > 0.0 && th < 1.0)) { kase = 1; break; }
        orc_xy_from_k(nc, z, K, th, x, y);
        orc_phase(&e, x, lx, NULL);
        orc_phase(&e, y, ly, NULL);
        for (int i = 0; i < nc; ++i) lnK[i] = lx[i] - ly[i];
        npre = k;
    }
    if (kase != 1 && kase != 4) {
        tpdx = 0.0; tpdy = 0.0;
        for (int i = 0; i < nc; ++i) {
            tpdx += x[i] * (log(x[i]) + lx[i] - d[i]);
            tpdy += y[i] * (log(y[i]) + ly[i] - d[i]);
        }
        double dG = (1.0 - th) * tpdx + th * tpdy;               /* R2 */
        kase = (tpdx < -o->eps_tm || tpdy < -o->eps_tm || dG < -o->eps_tm) ? 3 : 2;
    }
    /* R21: the composition with negative tangent-plane distance that proved
     * the instability: the triage phase with the smaller tpd (case 3), or
     * the stability trial the K re-estimate uses (below) */
    double wst[ORC_NCMAX];
    int have_w = 0;
    if (kase == 3) {
        for (int i = 0; i < nc; ++i) wst[i] = tpdx <= tpdy ? x[i] : y[i];
        have_w = 1;
    }
    res->info[ORC_I_CASE] = kase;
    res->info[ORC_I_PRE] = npre;
    /* the decisive value of a case-3 mixture: the most negative of the
     * triage's tpd(x), tpd(y) and Delta G */
    if (kase == 3) res->tm_dec = fmin(tpdx, fmin(tpdy, (1.0 - th) * tpdx + th * tpdy));

    /* Stability analysis (Sec. 2.2.1, Algorithm 2): vapour-like W = K z and
     * liquid-like W = z / K from the Wilson K (R5), each by successive
     * substitution, then the second-order stand-in when not stopped. */
    double lnWt[2][ORC_NCMAX], tmt[2] = {INFINITY, INFINITY};
    int ran_sa = 0;
    int unstable = (kase == 3 || kase == 4);
    if (kase == 1 || kase == 2) {
        ran_sa = 1;
        for (int t = 0; t < 2; ++t) {
            for (int i = 0; i < nc; ++i) lnWt[t][i] = lnz[i] + (t == 0 ? lnKw[i] : -lnKw[i]);
            int nss = 0, nnt = 0;
            int out = orc_sa_ss(&e, d, lnWt[t], o, &nss, &tmt[t]);
            if (out == ORC_TRIAL_UNCONV)
                out = orc_sa_newton(&e, d, lnWt[t], o, o->tol_sa_tr, 1, &nnt, &tmt[t]);
            if (out == ORC_TRIAL_UNCONV) flags |= ORC_SA_UNCONV;
            res->info[t == 0 ? ORC_I_SS_V : ORC_I_SS_L] = nss;
            res->info[t == 0 ? ORC_I_NT_V : ORC_I_NT_L] = nnt;
            res->info[t == 0 ? ORC_I_OUT_V : ORC_I_OUT_L] = out;
        }
        unstable = (tmt[0] < -o->eps_tm) || (tmt[1] < -o->eps_tm);
        /* the decisive value after stability analysis: the smaller final tm */
        res->tm_dec = fmin(tmt[0], tmt[1]);
        if (unstable) {
            /* K re-estimate (Sec. 2.2.1, last paragraph) from the trial with
             * the smaller tm; a trial whose substitution diverged (tm not a
             * number) is never the one taken (R22) */
            const int ts = (tmt[1] < tmt[0] || isnan(tmt[0])) ? 1 : 0;
            if (ts == 1)
                for (int i = 0; i < nc; ++i) lnK[i] = lnz[i] - lnWt[1][i];
            else
                for (int i = 0; i < nc; ++i) lnK[i] = lnWt[0][i] - lnz[i];
            double sw = 0.0;
            for (int i = 0; i < nc; ++i) { wst[i] = exp(lnWt[ts][i]); sw += wst[i]; }
            for (int i = 0; i < nc; ++i) wst[i] /= sw;
            have_w = 1;
        }
    }

    /* min-TPD diagnostic: every trial run to full stationarity; tpd of each
     * non-trivial stationary composition, plus the triage tpd values. */
    if (o->want_min_tpd) {
        double mt = INFINITY;
        if (kase != 1) mt = fmin(mt, fmin(tpdx, tpdy));
        for (int t = 0; t < 2; ++t) {
            double lw[ORC_NCMAX], tmv;
            int ns, nn;
            if (ran_sa) memcpy(lw, lnWt[t], sizeof(double) * nc);
            else {
                for (int i = 0; i < nc; ++i) lw[i] = lnz[i] + (t == 0 ? lnKw[i] : -lnKw[i]);
                orc_opts o2 = *o; o2.eps_tm = INFINITY;
                orc_sa_ss(&e, d, lw, &o2, &ns, &tmv);
            }
            orc_opts o3 = *o; o3.max_newton = 400;
            orc_sa_newton(&e, d, lw, &o3, 1e-12, 0, &nn, &tmv);
            if (!orc_is_trivial(nc, lw, z)) {
                double W[ORC_NCMAX];
                for (int i = 0; i < nc; ++i) W[i] = exp(lw[i]);
                mt = fmin(mt, orc_tpd(&e, W, d));
            }
        }
        res->min_tpd = mt;
    }

    res->info[ORC_I_UNSTABLE] = unstable;
    if (o->decision_only) {
        /* the stability decision alone (Sec. 2.2.1 and 2.2.3): label 1 for a
         * mixture the flash would send to the phase split */
        res->label = unstable;
        res->info[ORC_I_FLAGS] = (int32_t)flags;
        return 0;
    }
    if (!unstable) {
        res->info[ORC_I_FLAGS] = (int32_t)flags;
        return 0;
    }

    /* Phase split: successive substitution, then the Newton stand-in and
     * refinement to the double-precision root (R8). */
    int conv = 0, rrf = 0;
    int nss = orc_split_ss(&e, z, lnK, o, &conv, &rrf);
    res->info[ORC_I_SS_SPLIT] = nss;
    res->info[ORC_I_SPLIT_SS_CONV] = conv;
    double thf, nV[ORC_NCMAX];
    for (int i = 0; i < nc; ++i) K[i] = exp(lnK[i]);
    const int no_root = rrf || orc_rr_solve(nc, z, K, &thf) != 0;
    if (no_root || !(thf > 0.0 && thf < 1.0)) {
        /* R21: the substitution left the two-phase region; restart from the
         * composition that proved the instability */
        if (!have_w || orc_split_restart(&e, z, d, wst, nV) != 0) {
            res->info[ORC_I_FLAGS] =
                (int32_t)(flags | (no_root ? ORC_RR_NO_ROOT : 0u) | ORC_SPLIT_FAILED);
            return 0;
        }
        flags |= ORC_SPLIT_RESTART;
    } else {
        orc_xy_from_k(nc, z, K, thf, x, y);
        for (int i = 0; i < nc; ++i) nV[i] = thf * y[i];
    }
    int nnt = 0;
    if (orc_split_newton(&e, z, nV, o, &nnt) != 0) flags |= ORC_SPLIT_UNCONV;
    double bv = 0.0;
    for (int i = 0; i < nc; ++i) bv += nV[i];
    const int degen1 = !(bv > 1e-10 && bv < 1.0 - 1e-10);
    const int triv1 = orc_split_is_trivial(nc, z, nV, bv);
    const int stalled = (flags & ORC_SPLIT_UNCONV) && fmin(bv, 1.0 - bv) < 1e-3;
    double nb[ORC_NCMAX];
    memcpy(nb, nV, sizeof(double) * nc);
    int restarted = 0;
    if ((degen1 || triv1 || stalled) && !(flags & ORC_SPLIT_RESTART) && have_w) {
        restarted = orc_split_restart(&e, z, d, wst, nV) == 0;
        /* no start below the feed's G: the first descent's point stands */
        if (!restarted) memcpy(nV, nb, sizeof(double) * nc);
    }
    if (restarted) {
        /* R21: the descent ended at a degenerate split, at the trivial point
         * (which an unstable feed's split cannot be: the composition w gives
         * a lower G) or stalled against the boundary (unconverged, a phase
         * below 1e-3 of the feed); restart once from the composition that
         * proved the instability */
        flags = (flags & ~ORC_SPLIT_UNCONV) | ORC_SPLIT_RESTART;
        int n2 = 0;
        if (orc_split_newton(&e, z, nV, o, &n2) != 0) flags |= ORC_SPLIT_UNCONV;
        nnt += n2;
        bv = 0.0;
        for (int i = 0; i < nc; ++i) bv += nV[i];
        if (stalled && !degen1 && !triv1 &&
            (!(bv > 1e-10 && bv < 1.0 - 1e-10) || orc_split_is_trivial(nc, z, nV, bv))) {
            /* the restarted descent failed: the stalled split is the result,
             * flagged unconverged */
            memcpy(nV, nb, sizeof(double) * nc);
            flags |= ORC_SPLIT_UNCONV;
            bv = 0.0;
            for (int i = 0; i < nc; ++i) bv += nV[i];
        }
    }
    res->info[ORC_I_NT_SPLIT] = nnt;
    /* a phase holding less than 1e-10 of the feed: degenerate split */
    if (!(bv > 1e-10 && bv < 1.0 - 1e-10)) {
        res->info[ORC_I_FLAGS] = (int32_t)(flags | ORC_SPLIT_FAILED);
        return 0;
    }
    double lkmax = 0.0, bl = 0.0;
    for (int i = 0; i < nc; ++i) bl += z[i] - nV[i];
    for (int i = 0; i < nc; ++i) {
        y[i] = nV[i] / bv;
        x[i] = (z[i] - nV[i]) / bl;
        double q = fabs(log(y[i] / x[i]));
        if (q > lkmax) lkmax = q;
    }
    if (lkmax < 1e-6) {
        res->info[ORC_I_FLAGS] = (int32_t)(flags | ORC_SPLIT_TRIVIAL);
        return 0;
    }
    /* R9: y is the phase with the larger compressibility factor */
    orc_phase_info px, py;
    orc_phase(&e, x, lx, &px);
    orc_phase(&e, y, ly, &py);
    int swap = px.Z > py.Z;
    res->info[ORC_I_NROOT_SWAP] = swap;
    res->label = 1;
    res->beta = swap ? 1.0 - bv : bv;
    for (int i = 0; i < nc; ++i) {
        res->x[i] = swap ? y[i] : x[i];
        res->y[i] = swap ? x[i] : y[i];
    }
    res->info[ORC_I_FLAGS] = (int32_t)flags;
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Exported entry points (loaded through ctypes by the test suite)         */
/* ---------------------------------------------------------------------- */

void orc_default_opts(orc_opts *o)
{
    o->max_pre_ss = 3;
    o->max_ss = 9;
    o->max_newton = 200;
    o->dem_every = 3;
    o->want_min_tpd = 0;
    o->max_newton_split = 200;
    o->tol_sa_ss = 1e-6;
    o->tol_sa_tr = 1e-6;
    o->tol_split_ss = 1e-8;
    o->tol_split = 1e-13;
    o->eps_tm = 1e-10;
    o->decision_only = 0;
}

int orc_ninfo(void) { return ORC_NINFO; }
int orc_ncmax(void) { return ORC_NCMAX; }

/* Batch driver over rows [begin, end).  props_per_mixture = 0: Tc, Pc, omega
 * hold nc values and kij nc*nc, shared by every mixture; 1: they hold n*nc
 * and n*nc*nc values, one set per mixture.  label/beta/x/y/min_tpd/tm/info are
 * full-size arrays indexed by mixture (min_tpd and tm may be NULL). */
void orc_flash_batch(int64_t n, int32_t nc, const double *z, const double *T,
                     const double *P, const double *Tc, const double *Pc,
                     const double *omega, const double *kij, int32_t props_per_mixture,
                     const double *lnk0, const int8_t *hint,
                     const orc_opts *o, int8_t *label, double *beta, double *x,
                     double *y, double *min_tpd, double *tm, int32_t *info, int64_t begin,
                     int64_t end)
{
    (void)n;
    orc_result r;
    for (int64_t m = begin; m < end; ++m) {
        const double *tc = props_per_mixture ? Tc + m * nc : Tc;
        const double *pc = props_per_mixture ? Pc + m * nc : Pc;
        const double *om = props_per_mixture ? omega + m * nc : omega;
        const double *kk = props_per_mixture ? kij + m * nc * nc : kij;
        orc_flash_one(nc, z + m * nc, T[m], P[m], tc, pc, om, kk, lnk0 ? lnk0 + m * nc : NULL,
                      hint ? (int)hint[m] : -1, o, &r);
        label[m] = (int8_t)r.label;
        beta[m] = r.beta;
        for (int i = 0; i < nc; ++i) { x[m * nc + i] = r.x[i]; y[m * nc + i] = r.y[i]; }
        if (min_tpd) min_tpd[m] = r.min_tpd;
        if (tm) tm[m] = r.tm_dec;
        if (info) memcpy(info + m * ORC_NINFO, r.info, sizeof(int32_t) * ORC_NINFO);
    }
}

/* Primitive probes for the self-tests. */
void orc_lnphi(int32_t nc, const double *Tc, const double *Pc, const double *omega,
               const double *kij, double T, double P, const double *c, double *lnphi,
               double *ABZ /* A, B, Z, nroots, r0, r1, r2 */)
{
    orc_eos e;
    orc_phase_info info;
    orc_eos_setup(nc, Tc, Pc, omega, kij, T, P, &e);
    orc_phase(&e, c, lnphi, &info);
    if (ABZ) {
        ABZ[0] = info.A; ABZ[1] = info.B; ABZ[2] = info.Z; ABZ[3] = info.nroots;
        ABZ[4] = info.roots[0]; ABZ[5] = info.roots[1]; ABZ[6] = info.roots[2];
    }
}

void orc_wilson_lnk(int32_t nc, const double *Tc, const double *Pc, const double *omega,
                    double T, double P, double *lnK)
{
    orc_wilson(nc, Tc, Pc, omega, T, P, lnK);
}

double orc_tpd_probe(int32_t nc, const double *Tc, const double *Pc, const double *omega,
                     const double *kij, double T, double P, const double *z,
                     const double *w)
{
    orc_eos e;
    double lp[ORC_NCMAX], d[ORC_NCMAX], zz[ORC_NCMAX], s = 0.0;
    orc_eos_setup(nc, Tc, Pc, omega, kij, T, P, &e);
    for (int i = 0; i < nc; ++i) s += z[i];
    for (int i = 0; i < nc; ++i) zz[i] = z[i] / s;
    orc_phase(&e, zz, lp, NULL);
    for (int i = 0; i < nc; ++i) d[i] = log(zz[i]) + lp[i];
    return orc_tpd(&e, w, d);
}

/* Equal-fugacity residual at given vapour mole numbers (for the tests). */
double orc_split_residual(int32_t nc, const double *Tc, const double *Pc,
                          const double *omega, const double *kij, double T, double P,
                          const double *z, const double *nV, double *r)
{
    orc_eos e;
    double G;
    orc_eos_setup(nc, Tc, Pc, omega, kij, T, P, &e);
    orc_split_res(&e, z, nV, r, &G);
    return G;
}

/* ---------------------------------------------------------------------- */
/* Dense Jacobian of a converged split (implicit function theorem)         */
/* ---------------------------------------------------------------------- */

/* Parameters p = (z_raw[nc], T, P, k_ab for a < b).  The split is the root
 * u of r(u; z~, T, P, k) = ln y + ln phi(y) - ln x - ln phi(x) = 0 (eq.
 * eq_cond in logarithms, eq. split_grad) with y = u / sum u and
 * x = (z~ - u) / sum(z~ - u), z~ = z_raw / sum z_raw; the outputs are
 * o = (beta = sum u, x, y).  By the implicit function theorem
 * du/dp = -(dr/du)^-1 dr/dp.  The partial Jacobians dr/du and dr/d(z~, T,
 * P, k) are fourth-order central differences (f(-2h), f(-h), f(h), f(2h);
 * steps of hrel relative to the smallest quantity they move: u_j and the
 * liquid moles z~ - u for u and z~); dr/dz
 * follows from dr/dz~ through the normalisation; the systems are solved by
 * Gaussian elimination; the outputs are differentiated in closed form:
 *   d beta = sum du, dy = (du - y d beta)/beta,
 *   dx = (dn^L - x sum dn^L)/(1 - beta), dn^L = dz~ - du. */

static void orc_res_zt(int nc, const double *u, const double *zt, double T, double P,
                       const double *Tc, const double *Pc, const double *omega,
                       const double *kij, double *r)
{
    orc_eos e;
    orc_eos_setup(nc, Tc, Pc, omega, kij, T, P, &e);
    orc_split_res(&e, zt, u, r, NULL);
}

/* J (row-major, (1+2nc) x (nc+2+nc(nc-1)/2)) of the outputs (beta, x, y) of a
 * converged two-phase result given in the library's orientation (y the
 * phase whose mole numbers are u = beta y).  Returns 0, or 1 when dr/du is
 * singular. */
int orc_flash_jacobian(int32_t nc, const double *zraw, double T, double P,
                       const double *Tc, const double *Pc, const double *omega,
                       const double *kij, double beta, const double *y, double hrel,
                       double *J)
{
    int np = nc + 2 + nc * (nc - 1) / 2, no = 1 + 2 * nc;
    double u[ORC_NCMAX], zt[ORC_NCMAX], s = 0.0, nlmin = INFINITY;
    double Ju[ORC_NCMAX * ORC_NCMAX], rp[ORC_NCMAX], rm[ORC_NCMAX], ut[ORC_NCMAX];
    double Jz[ORC_NCMAX * ORC_NCMAX], zp[ORC_NCMAX];
    for (int i = 0; i < nc; ++i) s += zraw[i];
    for (int i = 0; i < nc; ++i) {
        zt[i] = zraw[i] / s;
        u[i] = beta * y[i];
        nlmin = fmin(nlmin, zt[i] - u[i]);
    }
    double r2p[ORC_NCMAX], r2m[ORC_NCMAX];
    for (int j = 0; j < nc; ++j) {
        double h = hrel * fmin(u[j], zt[j] - u[j]);
        memcpy(ut, u, sizeof(double) * nc);
        ut[j] = u[j] + h; orc_res_zt(nc, ut, zt, T, P, Tc, Pc, omega, kij, rp);
        ut[j] = u[j] - h; orc_res_zt(nc, ut, zt, T, P, Tc, Pc, omega, kij, rm);
        ut[j] = u[j] + 2.0 * h; orc_res_zt(nc, ut, zt, T, P, Tc, Pc, omega, kij, r2p);
        ut[j] = u[j] - 2.0 * h; orc_res_zt(nc, ut, zt, T, P, Tc, Pc, omega, kij, r2m);
        for (int i = 0; i < nc; ++i)
            Ju[i * nc + j] = (8.0 * (rp[i] - rm[i]) - (r2p[i] - r2m[i])) / (12.0 * h);
    }
    /* dr/dz~_k */
    for (int k = 0; k < nc; ++k) {
        double h = hrel * fmin(zt[k] - u[k], nlmin * 1e3);
        memcpy(zp, zt, sizeof(double) * nc);
        zp[k] = zt[k] + h; orc_res_zt(nc, u, zp, T, P, Tc, Pc, omega, kij, rp);
        zp[k] = zt[k] - h; orc_res_zt(nc, u, zp, T, P, Tc, Pc, omega, kij, rm);
        zp[k] = zt[k] + 2.0 * h; orc_res_zt(nc, u, zp, T, P, Tc, Pc, omega, kij, r2p);
        zp[k] = zt[k] - 2.0 * h; orc_res_zt(nc, u, zp, T, P, Tc, Pc, omega, kij, r2m);
        for (int i = 0; i < nc; ++i)
            Jz[i * nc + k] = (8.0 * (rp[i] - rm[i]) - (r2p[i] - r2m[i])) / (12.0 * h);
    }
    double k2[ORC_NCMAX * ORC_NCMAX], drp[ORC_NCMAX], du[ORC_NCMAX], dzt[ORC_NCMAX];
    double M[ORC_NCMAX * ORC_NCMAX];
    int pa = 0, pb = 0;
    for (int q = 0; q < np; ++q) {
        for (int i = 0; i < nc; ++i) dzt[i] = 0.0;
        if (q < nc) {
            /* dz~/dz_q = (e_q - z~)/sum z */
            for (int i = 0; i < nc; ++i) dzt[i] = ((i == q ? 1.0 : 0.0) - zt[i]) / s;
            for (int i = 0; i < nc; ++i) {
                double a = 0.0;
                for (int k = 0; k < nc; ++k) a += Jz[i * nc + k] * dzt[k];
                drp[i] = a;
            }
        } else if (q == nc || q == nc + 1) {
            double h = hrel * (q == nc ? T : P);
            double dT = q == nc ? h : 0.0, dP = q == nc + 1 ? h : 0.0;
            orc_res_zt(nc, u, zt, T + dT, P + dP, Tc, Pc, omega, kij, rp);
            orc_res_zt(nc, u, zt, T - dT, P - dP, Tc, Pc, omega, kij, rm);
            orc_res_zt(nc, u, zt, T + 2.0 * dT, P + 2.0 * dP, Tc, Pc, omega, kij, r2p);
            orc_res_zt(nc, u, zt, T - 2.0 * dT, P - 2.0 * dP, Tc, Pc, omega, kij, r2m);
            for (int i = 0; i < nc; ++i)
                drp[i] = (8.0 * (rp[i] - rm[i]) - (r2p[i] - r2m[i])) / (12.0 * h);
        } else {
            /* symmetric perturbation of k_ab = k_ba */
            if (q == nc + 2) { pa = 0; pb = 1; }
            else if (++pb == nc) { ++pa; pb = pa + 1; }
            double h = hrel;
            const double steps[4] = {h, -h, 2.0 * h, -2.0 * h};
            double *outs[4] = {rp, rm, r2p, r2m};
            for (int t = 0; t < 4; ++t) {
                memcpy(k2, kij, sizeof(double) * nc * nc);
                k2[pa * nc + pb] += steps[t];
                k2[pb * nc + pa] += steps[t];
                orc_res_zt(nc, u, zt, T, P, Tc, Pc, omega, k2, outs[t]);
            }
            for (int i = 0; i < nc; ++i)
                drp[i] = (8.0 * (rp[i] - rm[i]) - (r2p[i] - r2m[i])) / (12.0 * h);
        }
        for (int i = 0; i < nc; ++i) du[i] = -drp[i];
        memcpy(M, Ju, sizeof(double) * nc * nc);
        if (orc_gepp(nc, M, du)) return 1;
        double db = 0.0, dnl = 0.0;
        for (int i = 0; i < nc; ++i) { db += du[i]; dnl += dzt[i] - du[i]; }
        J[0 * np + q] = db;
        for (int i = 0; i < nc; ++i) {
            double xi = (zt[i] - u[i]) / (1.0 - beta);
            J[(1 + i) * np + q] = ((dzt[i] - du[i]) - xi * dnl) / (1.0 - beta);
            J[(1 + nc + i) * np + q] = (du[i] - y[i] * db) / beta;
        }
    }
    (void)no;
    return 0;
}
