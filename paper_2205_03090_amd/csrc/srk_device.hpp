// srk_device.hpp -- per-lane SRK phase model, Rachford-Rice solve and dense
// trust-region kernels for gfx950, in FP64, one mixture per lane with the
// component count NC fixed at compile time so that every per-component array
// lives in VGPRs.
//
// Sources: SRK mixing/combining rules, cubic in Z, Halley iteration with
// deflation and fugacity coefficients (Appendix A); Rachford-Rice equation
// and the Leibovici-Neoschil helper function (eq. RR, Appendix C); trust-
// region steps of Hebden type (Appendix B).  The composition derivatives of
// ln phi are not printed in the paper; they are derived here from eq. lnphi
// (see phase_derivs).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ptf {

// SRK constants as printed with the combining rules (Appendix A, eqs. a_i, b_i)
// and the Wilson correlation coefficient (Sec. 2.2.1, eq. wilson).
constexpr double kOmegaA = 0.42748;
constexpr double kOmegaB = 0.08664;
constexpr double kWilson = 5.373;

template <int NC>
struct Tri {
    static constexpr int N = NC * (NC + 1) / 2;
};
__host__ __device__ constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// Algorithmic flop counts (FMA = 2; add, mul, div, sqrt, exp, log = 1 each)
// of the primitives below, accumulated per mixture.
template <int NC>
struct Cost {
    static constexpr uint32_t mix = 2 * NC + 1 + NC + NC + 2 * NC * (NC - 1) + 4 * NC;
    static constexpr uint32_t halley = 17;
    static constexpr uint32_t deflate = 12;
    static constexpr uint32_t polish = 9;
    static constexpr uint32_t gibbs = 8;
    static constexpr uint32_t lnphi = 8 + 5 * NC;
    static constexpr uint32_t derivs = 30 * NC + 9 * (NC * (NC + 1) / 2) + 6;
    static constexpr uint32_t rr_iter = 6 * NC + 12;
    static constexpr uint32_t chol = (NC * (NC - 1) * (NC + 1)) / 3 + 2 * NC + NC * (NC + 1);
    static constexpr uint32_t trisolve = 2 * NC * NC;
};

// Per-lane constants of one mixture: s_i = sqrt(A_i) and B_i, both scaled by
// P/(RT)^2 and P/(RT), in which form the gas constant cancels:
// A_i = OMEGA_A alpha_i (Tc_i/T)^2 P/Pc_i, B_i = OMEGA_B (Tc_i/T) P/Pc_i.
template <int NC>
struct Eos {
    double s[NC];
    double b[NC];
};

template <int NC>
__device__ __forceinline__ void eos_setup(Eos<NC> &e, const double *__restrict__ Tc,
                                          const double *__restrict__ Pc,
                                          const double *__restrict__ om, double T, double P)
{
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        const double w = om[i];
        const double m = 0.480 + 1.574 * w - 0.176 * w * w;
        const double a = 1.0 + m * (1.0 - sqrt(T / Tc[i]));
        const double tr = Tc[i] / T;
        const double pr = P / Pc[i];
        // sqrt(OMEGA_A alpha tr^2 pr) = |a| tr sqrt(OMEGA_A pr)
        e.s[i] = fabs(a) * tr * sqrt(kOmegaA * pr);
        e.b[i] = kOmegaB * tr * pr;
    }
}

// Output of one phase evaluation E(c).
template <int NC>
struct Phase {
    double psi[NC];    // psi'_i = sum_j (1 - k_ij) s_j c_j, so psi_i = s_i psi'_i
    double lnphi[NC];
    double A, B, Z, L, lzb, q1, q2;
    int nroots;
};

// Minimum-Gibbs root of Z^3 - Z^2 + (A - B - B^2) Z - AB = 0 (eq. cubic_Z).
// Halley's iteration (eq. halley) from the liquid-like start Z = B (or from
// zs, the root chosen at the previous iterate of the same phase, when it lies
// inside the bracket: deflation recovers the other roots from whichever root
// the iteration reaches, so the root set and the choice below do not depend
// on the start), kept
// inside the sign-change bracket [B, 1+B] (f(B) = -2B^2 < 0, f(1+B) = A > 0),
// stopping when a Halley step is below 1e-8 Z or at an exact zero of f;
// deflation to a quadratic for the other
// roots; physical roots are those above B; each kept root gets one Newton
// correction on the full cubic; between the smallest (liquid) and largest
// (vapour) root the one with the lower reduced residual Gibbs energy
// g = Z - 1 - ln(Z - B) - (A/B) ln(1 + B/Z) is kept (ties go to the liquid).
__device__ __forceinline__ void cubic_root(double A, double B, double &Zout, double &Lout,
                                           double &lzbout, int &nroots, uint32_t &fl,
                                           double zs = -1.0)
{
    const double r1 = A - B * (1.0 + B);
    const double r0 = A * B;
    double lo = B, hi = 1.0 + B, Z = (zs > B && zs < 1.0 + B) ? zs : B;
    int it = 0;
    for (; it < 96; ++it) {
        const double f = ((Z - 1.0) * Z + r1) * Z - r0;
        if (f == 0.0) break;   // Z is a root
        const double fp = (3.0 * Z - 2.0) * Z + r1;
        const double fpp = 6.0 * Z - 2.0;
        if (f < 0.0) lo = Z; else hi = Z;
        const double Zn = Z - (2.0 * f * fp) / (2.0 * fp * fp - f * fpp);
        // the paper's test |Z_new/Z - 1| < 1e-8 on the Halley step.  It is
        // taken before the bracket test: at the root to rounding the step is
        // zero and lands on the end point just moved to Z, which must count
        // as converged, not as a step leaving the bracket (bisecting from
        // there walks back to the root one bit per iteration).
        if (fabs(Zn - Z) < 1e-8 * Z) {
            Z = fmin(fmax(Zn, lo), hi);
            break;
        }
        // a small bisection step says nothing about the distance to the root,
        // so only Halley steps are tested
        Z = (Zn > lo && Zn < hi) ? Zn : 0.5 * (lo + hi);
        if (!(hi - lo > 0.0)) break;
    }
    fl += Cost<1>::halley * (uint32_t)(it + 1);
    // deflation f = (Z - Z0)(Z^2 + p Z + q)
    const double p = Z - 1.0;
    const double q = p * Z + r1;
    const double disc = p * p - 4.0 * q;
    double zl = Z, zv = Z;
    nroots = 1;
    fl += Cost<1>::deflate;
    if (disc >= 0.0) {
        const double sq = sqrt(disc);
        const double t = -0.5 * (p + copysign(sq, p));
        const double ra = t;
        const double rb = (t != 0.0) ? q / t : -p;
        if (ra > B) { zl = fmin(zl, ra); zv = fmax(zv, ra); ++nroots; }
        if (rb > B) { zl = fmin(zl, rb); zv = fmax(zv, rb); ++nroots; }
    }
    // Newton correction on the full cubic (kept only when small)
    auto pol = [&](double z0) {
        const double f = ((z0 - 1.0) * z0 + r1) * z0 - r0;
        const double fp = (3.0 * z0 - 2.0) * z0 + r1;
        const double d = f / fp;
        return (fabs(d) < 1e-3 * z0) ? z0 - d : z0;
    };
    if (nroots > 1) {
        zl = pol(zl);
        zv = pol(zv);
        fl += 2 * Cost<1>::polish;
        const double lzl = log(zl - B), ll = log1p(B / zl);
        const double lzv = log(zv - B), lv = log1p(B / zv);
        const double ab = A / B;
        const double gl = zl - 1.0 - lzl - ab * ll;
        const double gv = zv - 1.0 - lzv - ab * lv;
        fl += 2 * Cost<1>::gibbs;
        if (gv < gl) { Zout = zv; Lout = lv; lzbout = lzv; }
        else { Zout = zl; Lout = ll; lzbout = lzl; }
    } else {
        Z = pol(Z);
        fl += Cost<1>::polish + 4;
        Zout = Z;
        Lout = log1p(B / Z);
        lzbout = log(Z - B);
    }
}

// Fugacity coefficients of one phase (eq. lnphi) for mole numbers w (any
// positive scale).  With t_i = s_i c_i and S = sum t:
//   psi'_i = S - sum_{j != i} k_ij t_j,   A = sum t_i psi'_i,   B = sum c_i B_i,
//   ln phi_i = B_i q1 - ln(Z - B) - q2 s_i psi'_i,
//   q1 = (Z - 1 + (A/B) L)/B,  q2 = 2L/B,  L = ln(1 + B/Z).
// K points at the shared nc*nc k_ij table (compile-time indexed, so that the
// loads are wave-uniform).
template <int NC>
__device__ __forceinline__ void phase_eval(Phase<NC> &o, const Eos<NC> &e,
                                           const double *__restrict__ K, const double (&w)[NC],
                                           uint32_t &fl, double zs = -1.0)
{
    double sum = 0.0;
#pragma unroll
    for (int i = 0; i < NC; ++i) sum += w[i];
    const double inv = 1.0 / sum;
    double c[NC], t[NC], S = 0.0;
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        c[i] = w[i] * inv;
        t[i] = e.s[i] * c[i];
        S += t[i];
    }
#pragma unroll
    for (int i = 0; i < NC; ++i) o.psi[i] = S;
#pragma unroll
    for (int i = 1; i < NC; ++i)
#pragma unroll
        for (int j = 0; j < i; ++j) {
            const double k = K[i * NC + j];
            o.psi[i] -= k * t[j];
            o.psi[j] -= k * t[i];
        }
    double A = 0.0, B = 0.0;
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        A += t[i] * o.psi[i];
        B += c[i] * e.b[i];
    }
    fl += Cost<NC>::mix;
    cubic_root(A, B, o.Z, o.L, o.lzb, o.nroots, fl, zs);
    o.A = A;
    o.B = B;
    const double ib = 1.0 / B;
    o.q1 = (o.Z - 1.0 + A * ib * o.L) * ib;
    o.q2 = 2.0 * o.L * ib;
#pragma unroll
    for (int i = 0; i < NC; ++i) o.lnphi[i] = e.b[i] * o.q1 - o.lzb - o.q2 * e.s[i] * o.psi[i];
    fl += Cost<NC>::lnphi;
}

// Unit-mole composition derivatives Phi_ij = n d ln phi_i / d n_j at fixed
// T, P, lower triangle only (Phi is symmetric: it is the Hessian of n g_res).
// With D_j(.) = n d(.)/d n_j:
//   D_j A = 2 (s_j psi'_j - A),  D_j B = B_j - B,
//   D_j Z = -(f_A D_j A + f_B D_j B)/f_Z  (implicit differentiation of the
//           cubic: f_A = Z - B, f_B = -(1+2B) Z - A, f_Z = 3Z^2 - 2Z + A - B - B^2),
//   D_j L = (Z D_j B - B D_j Z)/(Z (Z + B)),  D_j psi'_i = (1-k_ij) s_j - psi'_i,
// and differentiating ln phi_i = B_i q1 - ln(Z - B) - q2 s_i psi'_i:
//   Phi_ij = B_i D_j q1 - D_j ln(Z-B) - s_i psi'_i D_j q2
//            + q2 s_i psi'_i - q2 s_i (1 - k_ij) s_j.
template <int NC>
__device__ __forceinline__ void phase_derivs(double (&Phi)[Tri<NC>::N], const Phase<NC> &o,
                                             const Eos<NC> &e, const double *__restrict__ K,
                                             uint32_t &fl)
{
    const double A = o.A, B = o.B, Z = o.Z, L = o.L;
    const double fA = Z - B;
    const double fB = -(1.0 + 2.0 * B) * Z - A;
    const double fZ = (3.0 * Z - 2.0) * Z + A - B - B * B;
    const double ifZ = 1.0 / fZ;
    const double ib = 1.0 / B;
    const double izzb = 1.0 / (Z * (Z + B));
    const double izb = 1.0 / (Z - B);
    double al[NC], be[NC], ga[NC], sp[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j) {
        sp[j] = e.s[j] * o.psi[j];
        const double dA = 2.0 * (sp[j] - A);
        const double dB = e.b[j] - B;
        const double dZ = -(fA * dA + fB * dB) * ifZ;
        const double dL = (Z * dB - B * dZ) * izzb;
        be[j] = (dZ - dB) * izb;
        ga[j] = 2.0 * (dL - L * dB * ib) * ib;
        al[j] = (dZ + (dA * L + A * dL) * ib - A * L * dB * ib * ib) * ib - o.q1 * dB * ib;
    }
#pragma unroll
    for (int i = 0; i < NC; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            const double kap = (i == j) ? 1.0 : 1.0 - K[i * NC + j];
            Phi[tri(i, j)] = e.b[i] * al[j] - be[j] - sp[i] * ga[j] + o.q2 * sp[i]
                             - o.q2 * e.s[i] * kap * e.s[j];
        }
    fl += Cost<NC>::derivs;
}

// Rachford-Rice root (eq. RR) by the Leibovici-Neoschil method (Appendix C):
// Newton on h(th) = (th - a_l)(a_r - th) f_RR(th), a_l = 1/(1 - Kmax),
// a_r = 1/(1 - Kmin), with bisection whenever the Newton step leaves the
// shrinking bracket of the root; stops when a Newton step is below 1e-8.
// Returns false when all K lie on one side of 1 (no root in the window).
template <int NC>
__device__ __forceinline__ bool rr_solve(const double (&z)[NC], const double (&K)[NC],
                                         double &th, uint32_t &fl)
{
    double kmax = K[0], kmin = K[0];
#pragma unroll
    for (int i = 1; i < NC; ++i) { kmax = fmax(kmax, K[i]); kmin = fmin(kmin, K[i]); }
    if (!(kmax > 1.0) || !(kmin < 1.0)) return false;
    const double al = 1.0 / (1.0 - kmax), ar = 1.0 / (1.0 - kmin);
    double lo = al, hi = ar;
    double t = (th > al && th < ar) ? th : 0.5;
    int it = 0;
    for (; it < 200; ++it) {
        double f = 0.0, fp = 0.0;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            const double c = K[i] - 1.0;
            const double r = 1.0 / (1.0 + c * t);
            const double u = z[i] * c * r;
            f += u;
            fp -= u * c * r;
        }
        if (f > 0.0) lo = t; else hi = t;
        const double da = t - al, db = ar - t;
        const double h = da * db * f;
        const double hp = (db - da) * f + da * db * fp;
        const double tn = t - h / hp;
        // converged Newton step (tested before the bracket test, for the
        // same reason as in cubic_root: at the root the step is zero and
        // lands on the end point just moved to t)
        if (fabs(tn - t) < 1e-8) {
            t = fmin(fmax(tn, lo), hi);
            break;
        }
        t = (tn > lo && tn < hi) ? tn : 0.5 * (lo + hi);
        if (!(hi - lo > 0.0)) break;
    }
    fl += Cost<NC>::rr_iter * (uint32_t)(it + 1);
    th = t;
    return true;
}

// ---------------------------------------------------------------------------
// Dense symmetric kernels on packed lower triangles (row-major, tri(i,j)).
// ---------------------------------------------------------------------------

// Cholesky factor of H + shift*I into Lf (diagonal entries stored as
// reciprocals in dinv as well).  Returns false when a pivot is not positive.
template <int NC>
__device__ __forceinline__ bool cholesky(double (&Lf)[Tri<NC>::N], double (&dinv)[NC],
                                         const double (&H)[Tri<NC>::N], double shift,
                                         uint32_t &fl)
{
    bool ok = true;
#pragma unroll
    for (int i = 0; i < NC; ++i) {
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            double s = H[tri(i, j)] + ((i == j) ? shift : 0.0);
#pragma unroll
            for (int k = 0; k < j; ++k) s -= Lf[tri(i, k)] * Lf[tri(j, k)];
            if (i == j) {
                ok = ok && (s > 0.0);
                const double d = sqrt(fmax(s, 1e-300));
                Lf[tri(i, i)] = d;
                dinv[i] = 1.0 / d;
            } else {
                Lf[tri(i, j)] = s * dinv[j];
            }
        }
    }
    fl += Cost<NC>::chol;
    return ok;
}

// Solves L y = b (forward substitution).
template <int NC>
__device__ __forceinline__ void lower_solve(double (&y)[NC], const double (&Lf)[Tri<NC>::N],
                                            const double (&dinv)[NC], const double (&b)[NC])
{
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        double s = b[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= Lf[tri(i, k)] * y[k];
        y[i] = s * dinv[i];
    }
}

// Solves L^T x = y (back substitution).
template <int NC>
__device__ __forceinline__ void upper_solve(double (&x)[NC], const double (&Lf)[Tri<NC>::N],
                                            const double (&dinv)[NC], const double (&y)[NC])
{
#pragma unroll
    for (int i = NC - 1; i >= 0; --i) {
        double s = y[i];
#pragma unroll
        for (int k = i + 1; k < NC; ++k) s -= Lf[tri(k, i)] * x[k];
        x[i] = s * dinv[i];
    }
}

template <int NC>
__device__ __forceinline__ double norm2(const double (&v)[NC])
{
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NC; ++i) s += v[i] * v[i];
    return sqrt(s);
}

// Trust-region step of Hebden type (Appendix B): u solves (H + eta I) u = -g
// with eta >= 0 such that H + eta I is positive definite and ||u|| <= radius;
// when the unshifted Newton step is inside the region it is taken (eta = 0).
// Otherwise eta is found in the bracket [max(0, -min H_ii),
// ||g||/radius + max_i sum_j |H_ij|] (the upper end makes ||u|| <= radius):
// when H is positive definite the search starts with the Newton update of
// eta from 0 (using the factor of H already computed), otherwise at the lower
// end (or 1e-3 of the upper end); a failed factorisation raises the lower
// end and moves eta to the geometric mean of the bracket; a successful one
// takes a Newton step on Hebden's
// secular equation 1/||u(eta)|| = 1/radius, kept inside the bracket; ||u|| within
// 10 % of the radius is accepted; at most 12 factorisations.  If no shift
// succeeds, the Cauchy point (steepest descent minimising the model inside the
// region) is returned.  radius <= 0 on entry asks for the initial radius:
// ||Newton step|| when H is positive definite, else 1.  Returns the predicted
// change of the quadratic model g.u + u'Hu/2 (negative) and whether the step
// is the unshifted Newton step; Lf then holds the factor of H.  With
// newton_only the call stops after the factorisation of H: eta0 tells
// whether H is positive definite, and u is the Newton step when it is.
template <int NC>
__device__ __forceinline__ double trust_step(double (&u)[NC], double &radius, bool &eta0,
                                             double (&Lf)[Tri<NC>::N], double (&dinv)[NC],
                                             const double (&H)[Tri<NC>::N],
                                             const double (&g)[NC], uint32_t &fl,
                                             bool newton_only = false)
{
    double mg[NC], y[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) mg[i] = -g[i];
    eta0 = false;
    bool have = false;
    double eta1 = -1.0;   // first shift from the eta = 0 factor, when positive definite
    if (cholesky<NC>(Lf, dinv, H, 0.0, fl)) {
        lower_solve<NC>(y, Lf, dinv, mg);
        upper_solve<NC>(u, Lf, dinv, y);
        fl += Cost<NC>::trisolve;
        const double nu = norm2<NC>(u);
        if (!(radius > 0.0)) radius = nu;
        if (nu <= radius) {
            eta0 = true;
            have = true;
        } else {
            // the Newton step leaves the region: the first Hebden update
            // starts from eta = 0 with the factor in hand
            double q[NC];
            lower_solve<NC>(q, Lf, dinv, u);
            const double nq = norm2<NC>(q);
            eta1 = (nu / nq) * (nu / nq) * (nu - radius) / radius;
            fl += NC * NC + 2 * NC + 6;
        }
    } else if (!(radius > 0.0)) {
        radius = 1.0;
    }
    if (newton_only) return 0.0;
    if (!have) {
        double hmin = H[0], rowmax = 0.0;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            hmin = fmin(hmin, H[tri(i, i)]);
            double r = 0.0;
#pragma unroll
            for (int j = 0; j < NC; ++j) r += fabs(H[i >= j ? tri(i, j) : tri(j, i)]);
            rowmax = fmax(rowmax, r);
        }
        double elo = fmax(0.0, -hmin);
        double ehi = norm2<NC>(g) / radius + rowmax;
        double eta = elo > 0.0 ? elo : 1e-3 * ehi;
        if (eta1 > 0.0 && eta1 < ehi) eta = eta1;
        for (int it = 0; it < 12; ++it) {
            if (!cholesky<NC>(Lf, dinv, H, eta, fl)) {
                elo = eta;
                eta = fmax(sqrt(elo * ehi), elo + 1e-3 * (ehi - elo));
                continue;
            }
            double ut[NC];
            lower_solve<NC>(y, Lf, dinv, mg);
            upper_solve<NC>(ut, Lf, dinv, y);
            fl += Cost<NC>::trisolve;
            const double nu = norm2<NC>(ut);
#pragma unroll
            for (int i = 0; i < NC; ++i) u[i] = ut[i];
            have = true;
            if (nu > 0.9 * radius && nu < 1.1 * radius) break;
            if (nu > radius) elo = eta; else ehi = eta;
            double q[NC];
            lower_solve<NC>(q, Lf, dinv, ut);
            const double nq = norm2<NC>(q);
            double en = eta + (nu / nq) * (nu / nq) * (nu - radius) / radius;
            if (!(en > elo && en < ehi)) en = fmax(sqrt(elo * ehi), elo + 1e-3 * (ehi - elo));
            eta = en;
        }
        if (!have) {
            // Cauchy point: -t g with t minimising the model on [0, radius/||g||]
            double gg = 0.0, ghg = 0.0;
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                gg += g[i] * g[i];
                double hg = 0.0;
#pragma unroll
                for (int j = 0; j < NC; ++j) hg += H[i >= j ? tri(i, j) : tri(j, i)] * g[j];
                ghg += g[i] * hg;
            }
            const double tmax = radius / sqrt(gg);
            const double t = (ghg > 0.0) ? fmin(gg / ghg, tmax) : tmax;
#pragma unroll
            for (int i = 0; i < NC; ++i) u[i] = -t * g[i];
            fl += 2 * NC * NC + 4 * NC;
        }
    }
    // predicted change g.u + u'Hu/2
    double gu = 0.0, uhu = 0.0;
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        gu += g[i] * u[i];
        double hu = 0.0;
#pragma unroll
        for (int j = 0; j < NC; ++j) hu += H[i >= j ? tri(i, j) : tri(j, i)] * u[j];
        uhu += u[i] * hu;
    }
    fl += 2 * NC * NC + 2 * NC;
    return gu + 0.5 * uhu;
}

}  // namespace ptf
