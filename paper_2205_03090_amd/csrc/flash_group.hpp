// flash_group.hpp -- the two trust-region stages (stability trials, SaTr;
// split, SpNt) with one group of G lanes per mixture, for the larger
// component counts.
//
// With one mixture per lane, a trust-region iteration keeps the packed
// Hessian, its Cholesky factor and the composition derivatives of two phases
// per lane: 3 nc(nc+1)/2 doubles, which at nc = 20 is several KB per lane and
// spills.  Here lane i of a group holds component i: its composition and
// gradient entries, row i of the Hessian and row i of the factor.  The
// Hessian row lives in the group's LDS region and the loops over it run
// rolled (a few iterations unrolled), so that it costs no registers; the
// factor row is kept both in LDS (the back substitution reads its columns)
// and in registers, where the factorisation and the forward substitution
// read it in unrolled loops.  Sums over components are butterfly
// reductions inside the group (every lane ends with the same bits:
// floating-point addition is commutative), vectors that every row needs are
// broadcast through the LDS region, and the back substitution reads the
// factor's columns there.  The
// mixture's scalars (cubic root, trust radius, counters, decisions) are
// computed identically in every lane of the group, so a group always takes
// one path.  The arithmetic is that of the per-lane items in flash_stages.hpp
// (Appendix B.1 and B.2, readings as listed there); only the order of the
// sums differs.
#pragma once

#include "flash_stages.hpp"

namespace ptf {

// Component counts from which the group variants are compiled.
constexpr int kGroupMinNc = 8;

// LDS doubles of one group: the factor and the Hessian (nc + 1 rows of LD
// doubles each: row i of L or of H, and a spare row that the lanes beyond nc
// write to) and five broadcast vectors of G entries.  The row stride
// LD = nc + 1 is odd, so that the lanes of a group, each reading its own row,
// fall in different banks.
template <int NC, int G>
struct GroupLds {
    static constexpr int LD = NC + 1;
    static constexpr int L = 0;
    static constexpr int H = (NC + 1) * LD;
    static constexpr int V = 2 * (NC + 1) * LD;
    static constexpr int N = V + 5 * G;
    // doubles of a group of an item with (kMatrix) or without the matrices
    template <class Item>
    static constexpr int of() { return Item::kMatrix ? N : 5 * G; }
};

// Orders the LDS accesses of one wavefront: stores before the fence are
// visible to the loads after it (the lanes of a group are in one wavefront).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int G>
__device__ __forceinline__ double gsum(double v)
{
#pragma unroll
    for (int o = 1; o < G; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int G>
__device__ __forceinline__ double gmax(double v)
{
#pragma unroll
    for (int o = 1; o < G; o <<= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

template <int G>
__device__ __forceinline__ double gmin(double v)
{
#pragma unroll
    for (int o = 1; o < G; o <<= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// Value of lane j of the caller's group.
__device__ __forceinline__ double gbcast(double v, int base, int j)
{
    return __shfl(v, base + j, 64);
}

// Lane geometry of a group and its LDS region.  The loops below over
// components j never test gi against j (such tests are loop-invariant lane
// masks that the compiler keeps live across the whole kernel): values of one
// lane are broadcast from it, results are read back from LDS slots, and the
// diagonal of a matrix row is carried separately.
template <int NC, int G>
struct Grp {
    // all five fields are set by the kernel before the first item begins
    int gi;       // component of this lane (valid below NC)
    int row;      // gi, or NC (the spare factor row) beyond the components
    int base;     // first lane of the group in the wavefront
    bool act;     // gi < NC
    double *sh;   // the group's region: GroupLds<NC, G>::of<Item>() doubles
    double *vb;   // its five broadcast vectors (after the matrices, if any)
    const double *ks;   // the block's kappa table in LDS (shared component set only)
    static constexpr int LD = GroupLds<NC, G>::LD;   // factor row stride
    __device__ __forceinline__ double *vec(int q) const { return vb + q * G; }
    __device__ __forceinline__ double *lsh() const { return sh + GroupLds<NC, G>::L; }
    // this lane's row of H = M + diag(dadd) without the addend (row NC
    // beyond the components)
    __device__ __forceinline__ double *hr() const { return sh + GroupLds<NC, G>::H + row * LD; }
};

// Row gi of the table kappa_ij = 1 - k_ij of the caller's mixture: for a
// shared component set a view of the block's table in LDS (loaded once per
// block), for one set per mixture the mixture's k row in global memory.
struct KapLds {
    // odd row stride: the lanes of a group, each on its own row, read
    // different banks
    template <int NC>
    static constexpr int stride() { return NC + 1; }
    const double *row;
    __device__ __forceinline__ double operator[](int j) const { return row[j]; }
};
struct KapGlobal {
    const double *krow;
    __device__ __forceinline__ double operator[](int j) const { return 1.0 - krow[j]; }
};

// Phase evaluation E(c) of one mixture across its group: this lane's share is
// component gi of the mole numbers w (0 on inactive lanes).  As phase_eval.
struct PhaseG {
    double A, B, Z, L, lzb, q1, q2;
    int nroots;
    double psi, lnphi;   // this lane's component
};

template <int NC, int G, class Kap>
__device__ __forceinline__ void phase_eval_g(PhaseG &o, const Grp<NC, G> &g, double s, double b,
                                             const Kap &kap, double w, uint32_t &fl, double zs)
{
    const double sum = gsum<G>(w);
    const double inv = 1.0 / sum;
    const double c = w * inv;
    const double t = s * c;
    double *tv = g.vec(0);
    tv[g.gi] = t;
    wave_lds_sync();
    double psi = 0.0;
#pragma unroll 4
    for (int j = 0; j < NC; ++j) psi += kap[j] * tv[j];
    wave_lds_sync();
    const double A = gsum<G>(g.act ? t * psi : 0.0);
    const double B = gsum<G>(c * b);
    fl += Cost<NC>::mix;
    cubic_root(A, B, o.Z, o.L, o.lzb, o.nroots, fl, zs);
    o.A = A;
    o.B = B;
    const double ib = 1.0 / B;
    o.q1 = (o.Z - 1.0 + A * ib * o.L) * ib;
    o.q2 = 2.0 * o.L * ib;
    o.psi = psi;
    o.lnphi = b * o.q1 - o.lzb - o.q2 * s * psi;
    fl += Cost<NC>::lnphi;
}

// Adds wrow * v_j * Phi_ij (row i = gi of Phi = n d ln phi / d n, as
// phase_derivs) to this lane's LDS row of H, entry j for every j (ACC
// false: stores it there), and the diagonal term to hdiag (the same bits as
// entry gi); v is this lane's entry of the scaling vector (0 on inactive
// lanes, where wrow is 0 too).
template <bool ACC, int NC, int G, class Kap>
__device__ __forceinline__ void phase_derivs_g(double &hdiag, const PhaseG &o,
                                               const Grp<NC, G> &g, double s, double b,
                                               const Kap &kap, double wrow, double v,
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
    const double sp = s * o.psi;
    const double dA = 2.0 * (sp - A);
    const double dB = b - B;
    const double dZ = -(fA * dA + fB * dB) * ifZ;
    const double dL = (Z * dB - B * dZ) * izzb;
    const double be = (dZ - dB) * izb;
    const double ga = 2.0 * (dL - L * dB * ib) * ib;
    const double al = (dZ + (dA * L + A * dL) * ib - A * L * dB * ib * ib) * ib - o.q1 * dB * ib;
    double *va = g.vec(0), *vb = g.vec(1), *vg = g.vec(2), *vs = g.vec(3), *vv = g.vec(4);
    va[g.gi] = al;
    vb[g.gi] = be;
    vg[g.gi] = ga;
    vs[g.gi] = s;
    vv[g.gi] = v;
    wave_lds_sync();
    const double cst = o.q2 * sp;
    const double qs = o.q2 * s;
    double *hr = g.hr();
#pragma unroll 4
    for (int j = 0; j < NC; ++j) {
        const double phi = b * va[j] - vb[j] - sp * vg[j] + cst - qs * kap[j] * vs[j];
        const double add = wrow * vv[j] * phi;
        hr[j] = ACC ? hr[j] + add : 0.0 + add;
    }
    wave_lds_sync();
    // kappa_ii = 1 - k_ii = 1 (a valid set has a zero diagonal)
    const double pd = b * al - be - sp * ga + cst - qs * 1.0 * s;
    hdiag += wrow * v * pd;
    fl += Cost<NC>::derivs;
}

// Cholesky factor of H + shift I, H = M + diag(dadd) with M given by the
// LDS rows (g.hr()) and dadd this lane's diagonal addend: the factor in the
// group's LDS, row gi by this lane (entries past the diagonal are not
// meaningful; the diagonal is written by lane j at step j), the same row in
// lr (registers: the loops over it run unrolled, so that a lane's own
// factor entries are register reads and each multiply-add reads one LDS
// value, broadcast), 1/L_ii of this row in dinv.  Returns whether every
// pivot was positive (the same in every lane).  As cholesky.
template <int NC, int G>
__device__ __forceinline__ bool chol_g(double (&lr)[NC], double &dinv, double dadd,
                                       double shift, const Grp<NC, G> &g, uint32_t &fl)
{
    constexpr int LD = Grp<NC, G>::LD;
    double *Ls = g.lsh();
    double *mine = Ls + g.row * LD;
    const double *hr = g.hr();
    bool ok = true;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
        double s = hr[j];
#pragma unroll
        for (int k = 0; k < j; ++k) s -= lr[k] * Ls[j * LD + k];
        // lane j's s is the pivot (before its diagonal terms)
        const double piv = gbcast(s + dadd, g.base, j) + shift;
        ok = ok && (piv > 0.0);
        const double d = sqrt(fmax(piv, 1e-300));
        const double dj = 1.0 / d;
        lr[j] = s * dj;
        mine[j] = lr[j];
        Ls[j * LD + j] = d;
        wave_lds_sync();
    }
    dinv = 1.0 / mine[g.act ? g.gi : 0];
    fl += Cost<NC>::chol;
    return ok;
}

// y = L^-1 b (forward substitution; this lane's entries of b and y, its
// factor row in lr).
template <int NC, int G>
__device__ __forceinline__ double lower_solve_g(const double (&lr)[NC], double dinv, double b,
                                                const Grp<NC, G> &g)
{
    double *yv = g.vec(1);
    double r = b;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
        const double yj = gbcast(r * dinv, g.base, j);
        yv[j] = yj;
        r -= lr[j] * yj;   // used by the lanes past j only
    }
    wave_lds_sync();
    const double y = yv[g.act ? g.gi : 0];
    wave_lds_sync();
    return g.act ? y : 0.0;
}

// x = L^-T y (back substitution, columns of L read from the LDS factor).
template <int NC, int G>
__device__ __forceinline__ double upper_solve_g(double dinv, double y, const Grp<NC, G> &g)
{
    const double *Ls = g.lsh();
    double *xv = g.vec(2);
    const int col = g.act ? g.gi : 0;
    double r = y;
#pragma unroll 2
    for (int k = NC - 1; k >= 0; --k) {
        const double xk = gbcast(r * dinv, g.base, k);
        xv[k] = xk;
        r -= Ls[k * Grp<NC, G>::LD + col] * xk;   // used by the lanes before k only
    }
    wave_lds_sync();
    const double x = xv[col];
    wave_lds_sync();
    return g.act ? x : 0.0;
}

// (H v)_i = sum_j M_ij v_j + dadd_i v_i from this lane's row and the group's v.
template <int NC, int G>
__device__ __forceinline__ double hv_g(double dadd, double v, const Grp<NC, G> &g)
{
    double *vv = g.vec(0);
    const double *hr = g.hr();
    vv[g.gi] = v;
    wave_lds_sync();
    double r = 0.0;
#pragma unroll 4
    for (int j = 0; j < NC; ++j) r += hr[j] * vv[j];
    wave_lds_sync();
    return r + dadd * v;
}

// Trust-region step of Hebden type across the group: as trust_step, with
// this lane's entries of u and g, row of M in LDS (g.hr()) and diagonal term
// (H = M + diag(dadd), M_ii = hdiag); the group's LDS holds the last factor,
// dinv this lane's 1/L_ii.  newton_only as in trust_step.
template <int NC, int G>
__device__ __forceinline__ double trust_step_g(double &u, double &radius, bool &eta0,
                                               double &dinv, double hdiag, double dadd,
                                               double gv, const Grp<NC, G> &g, uint32_t &fl,
                                               bool newton_only = false)
{
    double lr[NC];   // this lane's row of the last factor
    const double mg = -gv;
    eta0 = false;
    bool have = false;
    double eta1 = -1.0;
    u = 0.0;
    if (chol_g<NC, G>(lr, dinv, dadd, 0.0, g, fl)) {
        const double y = lower_solve_g<NC, G>(lr, dinv, mg, g);
        u = upper_solve_g<NC, G>(dinv, y, g);
        fl += Cost<NC>::trisolve;
        const double nu = sqrt(gsum<G>(u * u));
        if (!(radius > 0.0)) radius = nu;
        if (nu <= radius) {
            eta0 = true;
            have = true;
        } else {
            const double q = lower_solve_g<NC, G>(lr, dinv, u, g);
            const double nq = sqrt(gsum<G>(q * q));
            eta1 = (nu / nq) * (nu / nq) * (nu - radius) / radius;
            fl += NC * NC + 2 * NC + 6;
        }
    } else if (!(radius > 0.0)) {
        radius = 1.0;
    }
    if (newton_only) return 0.0;
    if (!have) {
        double rs = 0.0;
        const double *hr = g.hr();
#pragma unroll 4
        for (int j = 0; j < NC; ++j) rs += fabs(hr[j]);
        rs += fabs(hdiag + dadd) - fabs(hdiag);
        const double hmin = gmin<G>(g.act ? hdiag + dadd : INFINITY);
        const double rowmax = gmax<G>(g.act ? rs : 0.0);
        double elo = fmax(0.0, -hmin);
        double ehi = sqrt(gsum<G>(gv * gv)) / radius + rowmax;
        double eta = elo > 0.0 ? elo : 1e-3 * ehi;
        if (eta1 > 0.0 && eta1 < ehi) eta = eta1;
        for (int it = 0; it < 12; ++it) {
            if (!chol_g<NC, G>(lr, dinv, dadd, eta, g, fl)) {
                elo = eta;
                eta = fmax(sqrt(elo * ehi), elo + 1e-3 * (ehi - elo));
                continue;
            }
            const double y = lower_solve_g<NC, G>(lr, dinv, mg, g);
            const double ut = upper_solve_g<NC, G>(dinv, y, g);
            fl += Cost<NC>::trisolve;
            const double nu = sqrt(gsum<G>(ut * ut));
            u = ut;
            have = true;
            if (nu > 0.9 * radius && nu < 1.1 * radius) break;
            if (nu > radius) elo = eta; else ehi = eta;
            const double q = lower_solve_g<NC, G>(lr, dinv, ut, g);
            const double nq = sqrt(gsum<G>(q * q));
            double en = eta + (nu / nq) * (nu / nq) * (nu - radius) / radius;
            if (!(en > elo && en < ehi)) en = fmax(sqrt(elo * ehi), elo + 1e-3 * (ehi - elo));
            eta = en;
        }
        if (!have) {
            const double hg = hv_g<NC, G>(dadd, gv, g);
            const double gg = gsum<G>(gv * gv);
            const double ghg = gsum<G>(gv * hg);
            const double tmax = radius / sqrt(gg);
            const double t = (ghg > 0.0) ? fmin(gg / ghg, tmax) : tmax;
            u = -t * gv;
            fl += 2 * NC * NC + 4 * NC;
        }
    }
    const double hu = hv_g<NC, G>(dadd, u, g);
    const double gu = gsum<G>(gv * u);
    const double uhu = gsum<G>(u * hu);
    fl += 2 * NC * NC + 2 * NC;
    return gu + 0.5 * uhu;
}

// Row gi of the table kappa_ij = 1 - k_ij of mixture m (kappa_ii = 1: a
// valid set has a zero diagonal; the lanes beyond nc read row 0 and
// contribute nothing): the block's LDS table for a shared set, the
// mixture's row in registers for one set per mixture.
template <int NC, bool PM, int G>
__device__ __forceinline__ auto kappa_of(const Ctx<NC> &c, int64_t m, const Grp<NC, G> &g)
{
    const int row = g.act ? g.gi : 0;
    if constexpr (PM) {
        return KapGlobal{mix_props<NC, PM>(c.pr, m).K + row * NC};
    } else {
        return KapLds{g.ks + row * KapLds::stride<NC>()};
    }
}

// One substitution update with acceleration across the group (as
// ss_update): this lane's entries v, prev, s; returns ext.
template <int NC, int G>
__device__ __forceinline__ double ss_update_g(double &v, double &prev, double s, int u, int dem,
                                              uint32_t &fl)
{
    double ext = 0.0;
    if (dem > 0 && u >= 2 && (u % dem) == 0) {
        const double num = gsum<G>(s * s), den = gsum<G>(prev * s);
        const double lam = num / den;
        if (lam > 0.0 && lam < 1.0) ext = lam / (1.0 - lam);
        fl += 4 * NC + 3;
    }
    v += s + ext * s;
    prev = s;
    fl += 3 * NC;
    return ext;
}

// Rachford-Rice across the group (as rr_solve; this lane's z_i and K_i, 0
// and 1 on inactive lanes).  Every lane takes the same iterates.
template <int NC, int G>
__device__ __forceinline__ bool rr_solve_g(double z, double K, double &th, const Grp<NC, G> &g,
                                           uint32_t &fl)
{
    const double kmax = gmax<G>(g.act ? K : -INFINITY);
    const double kmin = gmin<G>(g.act ? K : INFINITY);
    if (!(kmax > 1.0) || !(kmin < 1.0)) return false;
    const double al = 1.0 / (1.0 - kmax), ar = 1.0 / (1.0 - kmin);
    double lo = al, hi = ar;
    double t = (th > al && th < ar) ? th : 0.5;
    const double c = K - 1.0;
    int it = 0;
    for (; it < 200; ++it) {
        const double r = 1.0 / (1.0 + c * t);
        const double u = z * c * r;
        const double f = gsum<G>(u);
        const double fp = -gsum<G>(u * c * r);
        if (f > 0.0) lo = t; else hi = t;
        const double da = t - al, db = ar - t;
        const double h = da * db * f;
        const double hp = (db - da) * f + da * db * fp;
        const double tn = t - h / hp;
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

// K -> Rachford-Rice -> normalised x, y across the group (as xy_from_lnk).
template <int NC, int G>
__device__ __forceinline__ bool xy_from_lnk_g(double &x, double &y, double lnk, double z,
                                              double &theta, const Grp<NC, G> &g, uint32_t &fl)
{
    const double K = g.act ? exp(lnk) : 1.0;
    fl += NC;
    if (!rr_solve_g<NC, G>(z, K, theta, g, fl)) return false;
    const double xr = z / (1.0 + theta * (K - 1.0));
    const double yr = K * xr;
    const double sx = gsum<G>(xr), sy = gsum<G>(yr);
    x = xr * (1.0 / sx);
    y = yr * (1.0 / sy);
    fl += 8 * NC + 2;
    return true;
}

// The feed normalised with the sum taken in component order (as load_z):
// this lane's z_i, 0 on inactive lanes.
template <int NC, int G>
__device__ __forceinline__ double load_z_g(const FlashArgs &a, int64_t m, const Grp<NC, G> &g)
{
    double sz = 0.0;
#pragma unroll
    for (int j = 0; j < NC; ++j) sz += a.z[m * NC + j];
    return g.act ? a.z[m * NC + g.gi] / sz : 0.0;
}

// ---------------------------------------------------------------------------
// SaSs with one group per trial (as SaSsItem)
// ---------------------------------------------------------------------------
template <int NC, bool PM, int G>
struct SaSsGroup {
    static constexpr int WAVES = 2;   // minimum wavefronts per SIMD
    static constexpr bool kPerMixture = PM;   // one component set per mixture
    static constexpr uint32_t OUT = 1u << L_SATR;   // lists the steps append to
    Outbox ob;   // list entries produced by the current step (lane gi = 0)
    static constexpr int LIST = L_SA;
    static constexpr int LIST2 = -1;
    static constexpr bool kMatrix = false;   // LDS: broadcast vectors only
    int64_t m;
    int t;
    double lw, prev, d, s, b;   // this lane's component
    double tmb, ext, zw;
    bool dem;
    int ss, steps;
    uint32_t fl, st;

    __device__ __forceinline__ bool begin(const Ctx<NC> &c, uint32_t id, const Grp<NC, G> &g)
    {
        m = id >> 1;
        t = (int)(id & 1u);
        const MixRec<NC> &r = c.rec[m];
        const int i = g.act ? g.gi : 0;
        s = g.act ? r.s[i] : 0.0;
        b = g.act ? r.b[i] : 0.0;
        d = g.act ? r.d[i] : 0.0;
        lw = g.act ? (t == 0 ? r.lnz[i] + r.lkw[i] : r.lnz[i] - r.lkw[i]) : 0.0;
        prev = 0.0;
        fl = 2 * NC;
        st = 0;
        ss = 0;
        steps = 0;
        dem = false;
        zw = -1.0;
        return true;
    }

    __device__ __forceinline__ void done(const Ctx<NC> &c, double tm, bool to_tr,
                                         const Grp<NC, G> &g)
    {
        MixRec<NC> &r = c.rec[m];
        if (g.act) r.lw[t][g.gi] = lw;
        if (g.gi == 0) {
            r.tm[t] = tm;
            r.it[t == 0 ? 1 : 3] = (int16_t)ss;
            r.it[t == 0 ? 2 : 4] = 0;
            r.tfl[t] = fl;
            r.tst[t] = st;
            if (to_tr) ob.put(L_SATR, (uint32_t)(2 * m + t));
        }
    }

    __device__ __forceinline__ bool step(const Ctx<NC> &c, const Grp<NC, G> &g)
    {
        const FlashArgs &a = c.a;
        const auto kap = kappa_of<NC, PM, G>(c, m, g);
        const double W = g.act ? exp(lw) : 0.0;
        fl += NC;
        PhaseG o;
        phase_eval_g<NC, G>(o, g, s, b, kap, W, fl, zw);
        zw = o.Z;
        const double grad = g.act ? lw + o.lnphi - d : 0.0;
        const double tm = 1.0 + gsum<G>(W * (grad - 1.0));
        const double gmx = gmax<G>(fabs(grad));
        fl += 6 * NC;
        if (tm < -a.eps_tm || gmx < a.tol_sa_ss) {
            done(c, tm, false, g);
            return true;
        }
        if (dem) {
            // an extrapolated point is kept only if it lowers tm
            dem = false;
            if (!(tm < tmb)) {
                lw -= ext * prev;
                if (++steps < kStepGuard) return false;
            }
        }
        if (ss < a.max_ss && ++steps < kStepGuard) {
            ext = ss_update_g<NC, G>(lw, prev, -grad, ss + 1, a.dem_every, fl);
            ++ss;
            if (ext > 0.0) {
                dem = true;
                tmb = tm;
            }
            return false;
        }
        // substitution budget spent: continue with the trust region
        done(c, tm, true, g);
        return true;
    }
};

// ---------------------------------------------------------------------------
// SpSs with one group per split (as SpSsItem)
// ---------------------------------------------------------------------------
template <int NC, bool PM, int G>
struct SpSsGroup {
    static constexpr int WAVES = 2;   // minimum wavefronts per SIMD
    static constexpr bool kPerMixture = PM;   // one component set per mixture
    static constexpr uint32_t OUT = (1u << L_NT) | (1u << L_NTP);
    Outbox ob;   // list entries produced by the current step (lane gi = 0)
    static constexpr int LIST = L_SPLIT;
    static constexpr int LIST2 = -1;
    static constexpr bool kMatrix = false;   // LDS: broadcast vectors only
    int64_t m;
    double z, lk, prev, s, b;   // this lane's component
    double theta, sgb, sext, zx, zy;
    bool dem;
    int ss, steps;
    uint32_t fl, status;

    __device__ __forceinline__ bool begin(const Ctx<NC> &c, uint32_t id, const Grp<NC, G> &g)
    {
        m = id;
        const MixRec<NC> &r = c.rec[m];
        const int i = g.act ? g.gi : 0;
        z = load_z_g<NC, G>(c.a, m, g);
        s = g.act ? r.s[i] : 0.0;
        b = g.act ? r.b[i] : 0.0;
        lk = g.act ? r.lk[i] : 0.0;
        prev = 0.0;
        theta = r.theta;
        fl = r.fl;
        status = r.status;
        ss = 0;
        steps = 0;
        dem = false;
        zx = zy = -1.0;
        return true;
    }

    __device__ __forceinline__ void fail(const Ctx<NC> &c, uint32_t bits, const Grp<NC, G> &g)
    {
        const FlashArgs &a = c.a;
        const MixRec<NC> &r = c.rec[m];
        if (g.act) {
            a.x[m * NC + g.gi] = z;
            a.y[m * NC + g.gi] = z;
        }
        if (g.gi == 0) {
            a.label[m] = 0;
            a.beta[m] = -1.0;
            if (a.iters) {
#pragma unroll
                for (int k = 0; k < 8; ++k) a.iters[m * 8 + k] = k == 5 ? (int16_t)ss : r.it[k];
            }
            if (a.status) a.status[m] = (uint16_t)(status | bits);
            if (a.flops) a.flops[m] = fl;
        }
    }

    // As SpSsItem::restart_or_fail.
    __device__ __forceinline__ void restart_or_fail(const Ctx<NC> &c, bool no_root,
                                                    uint32_t fail_bits, const Grp<NC, G> &g)
    {
        MixRec<NC> &r = c.rec[m];
        if (r.wsel < 0) {
            fail(c, kStSplitFailed | (no_root ? kStRrNoRoot : 0u) | fail_bits, g);
            return;
        }
        if (g.gi == 0) {
            r.rst = no_root ? 2 : 1;
            r.it[5] = (int16_t)ss;
            r.fl = fl;
            r.status = status | kStSplitTr | kStSplitRestart;
            ob.put(L_NT, (uint32_t)m);
        }
    }

    __device__ __forceinline__ bool step(const Ctx<NC> &c, const Grp<NC, G> &g)
    {
        const FlashArgs &a = c.a;
        const auto kap = kappa_of<NC, PM, G>(c, m, g);
        double x, y;
        if (!xy_from_lnk_g<NC, G>(x, y, lk, z, theta, g, fl)) {
            if (dem) {
                // an extrapolated point without a Rachford-Rice root is
                // rejected like one that does not lower G
                dem = false;
                lk -= sext * prev;
                if (++steps < kStepGuard) return false;
            }
            restart_or_fail(c, true, 0u, g);
            return true;
        }
        PhaseG o;
        phase_eval_g<NC, G>(o, g, s, b, kap, x, fl, zx);
        zx = o.Z;
        const double r0 = o.lnphi;
        phase_eval_g<NC, G>(o, g, s, b, kap, y, fl, zy);
        zy = o.Z;
        // G per unit feed (eq. gibbs) where an acceleration check needs it
        const bool dem_next = a.dem_every > 0 && ss + 1 >= 2 && ((ss + 1) % a.dem_every) == 0;
        double G_ = 0.0;
        if (dem || dem_next) {
            G_ = gsum<G>(g.act ? (1.0 - theta) * x * (log(x) + r0) + theta * y * (log(y) + o.lnphi)
                               : 0.0);
            fl += 10 * NC;
        }
        if (dem) {
            // an extrapolated point is kept only if it is a physical split and
            // lowers G
            dem = false;
            if (!(theta > 0.0 && theta < 1.0 && G_ < sgb)) {
                lk -= sext * prev;
                if (++steps < kStepGuard) return false;
            }
        }
        const double sv = g.act ? (r0 - o.lnphi) - lk : 0.0;
        const double dmax = gmax<G>(g.act ? fabs(exp(sv) - 1.0) : 0.0);
        fl += 4 * NC;
        const bool conv = dmax < a.tol_split_ss;
        const bool more = !conv && ss + 1 < a.max_ss && steps + 1 < kStepGuard;
        const double ext = ss_update_g<NC, G>(lk, prev, sv, ss + 1, more ? a.dem_every : 0, fl);
        ++ss;
        if (more) {
            ++steps;
            if (ext > 0.0) {
                dem = true;
                sgb = G_;
                sext = ext;
            }
            return false;
        }
        // hand over to the trust region: n^V = theta y from the final K
        MixRec<NC> &r = c.rec[m];
        if (!xy_from_lnk_g<NC, G>(x, y, lk, z, theta, g, fl)) {
            restart_or_fail(c, true, conv ? 0u : kStSplitTr, g);
            return true;
        }
        if (!(theta > 0.0 && theta < 1.0)) {
            restart_or_fail(c, false, conv ? 0u : kStSplitTr, g);
            return true;
        }
        if (g.act) r.lk[g.gi] = theta * y;
        if (g.gi == 0) {
            r.it[5] = (int16_t)ss;
            r.fl = fl;
            r.status = status | (conv ? 0u : kStSplitTr);
            ob.put(conv ? L_NTP : L_NT, (uint32_t)m);
        }
        return true;
    }
};

// ---------------------------------------------------------------------------
// SaTr with one group per trial (as SaTrItem)
// ---------------------------------------------------------------------------
template <int NC, bool PM, int G>
struct SaTrGroup {
    static constexpr int WAVES = 2;   // minimum wavefronts per SIMD
    static constexpr bool kPerMixture = PM;   // one component set per mixture
    static constexpr uint32_t OUT = 0u;
    static constexpr int LIST = L_SATR;
    static constexpr int LIST2 = -1;
    static constexpr bool kMatrix = true;   // LDS: Hessian and factor rows
    int64_t m;
    int t;
    double lw, lacc, d, s, b;   // this lane's component
    double rad, facc, pred, gacc, zw;
    double slen;   // length of the last step taken, in the region's norm
    bool pend;
    int tr, steps;
    uint32_t fl, st;

    __device__ __forceinline__ bool begin(const Ctx<NC> &c, uint32_t id, const Grp<NC, G> &g)
    {
        m = id >> 1;
        t = (int)(id & 1u);
        const MixRec<NC> &r = c.rec[m];
        const int i = g.act ? g.gi : 0;
        s = g.act ? r.s[i] : 0.0;
        b = g.act ? r.b[i] : 0.0;
        d = g.act ? r.d[i] : 0.0;
        lw = g.act ? r.lw[t][i] : 0.0;
        fl = r.tfl[t];
        st = r.tst[t];
        rad = 0.0;
        pend = false;
        tr = 0;
        steps = 0;
        zw = -1.0;
        return true;
    }

    __device__ __forceinline__ void done(const Ctx<NC> &c, double tm, const Grp<NC, G> &g)
    {
        MixRec<NC> &r = c.rec[m];
        if (g.act) r.lw[t][g.gi] = lw;
        if (g.gi == 0) {
            r.tm[t] = tm;
            r.it[t == 0 ? 2 : 4] = (int16_t)tr;
            r.tfl[t] = fl;
            r.tst[t] = st;
        }
    }

    __device__ __forceinline__ bool step(const Ctx<NC> &c, const Grp<NC, G> &g)
    {
        const FlashArgs &a = c.a;
        const auto kap = kappa_of<NC, PM, G>(c, m, g);
        const double W = g.act ? exp(lw) : 0.0;
        fl += NC;
        PhaseG o;
        phase_eval_g<NC, G>(o, g, s, b, kap, W, fl, zw);
        zw = o.Z;
        const double grad = g.act ? lw + o.lnphi - d : 0.0;
        const double tm = 1.0 + gsum<G>(W * (grad - 1.0));
        const double sw = gsum<G>(W);
        const double gv = sqrt(W) * grad;
        const double gmx = gmax<G>(fabs(gv));
        fl += 9 * NC;
        if (pend) {
            pend = false;
            bool accept;
            double ratio = 1.0;
            if (fabs(pred) < 1e-13) {
                accept = gmx < gacc;
            } else {
                ratio = (tm - facc) / pred;
                accept = (tm < facc) && ratio > 0.0;
            }
            // a rejected or poor step halves the radius, from the length of
            // the step taken when the boundary cut made it shorter
            if (!accept) {
                rad = 0.5 * fmin(rad, slen);
                lw = lacc;
                if (++steps < kStepGuard) return false;   // re-evaluate there
                st |= kStSaUnconv;
                done(c, facc, g);
                return true;
            }
            if (ratio <= 0.25) rad = 0.5 * fmin(rad, slen);
            else if (ratio >= 0.75) rad *= 2.0;
        }
        if (tm < -a.eps_tm || gmx < a.tol_sa_tr) {
            done(c, tm, g);
            return true;
        }
        if (tr >= a.max_tr_sa || ++steps >= kStepGuard) {
            st |= kStSaUnconv;
            done(c, tm, g);
            return true;
        }
        // H_ij = delta_ij (1 + grad_i/2) + sqrt(c_i c_j) Phi_ij
        const double rc = sqrt(W / sw);
        double hdiag = 0.0;
        phase_derivs_g<false>(hdiag, o, g, s, b, kap, rc, rc, fl);
        const double dadd = 1.0 + 0.5 * grad;
        fl += 2 * Tri<NC>::N + 4 * NC;
        double dinv = 0.0, u;
        bool eta0;
        double pr = trust_step_g<NC, G>(u, rad, eta0, dinv, hdiag, dadd, gv, g, fl);
        const double bi = 2.0 * sqrt(W);
        const double amax = gmin<G>((g.act && u < 0.0) ? fmin(1.0, 0.99 * bi / -u) : 1.0);
        slen = amax * sqrt(gsum<G>(g.act ? u * u : 0.0));
        if (amax < 1.0) {
            const double gu = gsum<G>(gv * u);
            pr = amax * gu + amax * amax * (pr - gu);
        }
        lacc = lw;
        if (g.act) lw = 2.0 * log(sqrt(W) + 0.5 * amax * u);
        fl += 6 * NC;
        facc = tm;
        gacc = gmx;
        pred = pr;
        pend = true;
        ++tr;
        return false;
    }
};

// ---------------------------------------------------------------------------
// SpNt with one group per split (as SpNtItem)
// ---------------------------------------------------------------------------
template <int NC, bool PM, int G>
struct SpNtGroup {
    static constexpr int WAVES = 2;   // minimum wavefronts per SIMD
    static constexpr bool kPerMixture = PM;   // one component set per mixture
    static constexpr uint32_t OUT = 0u;
    static constexpr int LIST = L_NT;
    static constexpr int LIST2 = L_NTP;
    static constexpr bool kMatrix = true;   // LDS: Hessian and factor rows
    static constexpr int NP = Tri<NC>::N;
    int64_t m;
    double z, v0, v1, s, b;   // this lane's component
    double srad, sfacc, spred, sgacc, sdprev, zx, zy;
    double slen;   // scaled length of the last trust-region step taken
    double sb, gf; // restart: current vapour amount of the start search, feed G
    bool tronly;   // refinement found H indefinite: take a trust-region step first
    bool spend, spol;
    bool start;    // restart: searching the start point (v1 holds the composition)
    bool restarted;
    bool back;     // the record holds a stalled first descent's n^V (r.lk)
    int tr, pol, steps, nhalf, rstk;
    int tr0;       // trust-region steps before a restart (each descent has the cap)
    uint32_t fl, status;

    // Restart of the split from the composition that proved the
    // instability (as SpNtItem::set_start).
    __device__ __forceinline__ void set_start(const MixRec<NC> &r, int rs, const Grp<NC, G> &g)
    {
        const double w = g.act ? exp(r.lw[r.wsel][g.gi]) : 0.0;
        const double sw = gsum<G>(w);
        v1 = w * (1.0 / sw);
        const double bmax = fmin(1.0, gmin<G>(g.act ? z / v1 : 1.0));
        gf = gsum<G>(g.act ? z * r.d[g.gi] : 0.0);
        sb = 0.5 * bmax;
        v0 = sb * v1;
        fl += 6 * NC + 2;
        start = restarted = true;
        nhalf = 0;
        rstk = rs;
        tr0 = tr;
        steps = 0;   // the restart happens once: the item stays bounded
        srad = 0.0;
        spend = spol = tronly = false;
        zx = zy = -1.0;
    }

    __device__ __forceinline__ bool begin(const Ctx<NC> &c, uint32_t id, const Grp<NC, G> &g)
    {
        m = id;
        const MixRec<NC> &r = c.rec[m];
        const int i = g.act ? g.gi : 0;
        // the feed normalised with the sum taken in component order, as load_z
        double sz = 0.0;
#pragma unroll
        for (int j = 0; j < NC; ++j) sz += c.a.z[m * NC + j];
        z = g.act ? c.a.z[m * NC + i] / sz : 0.0;
        s = g.act ? r.s[i] : 0.0;
        b = g.act ? r.b[i] : 0.0;
        v0 = g.act ? r.lk[i] : 0.0;
        v1 = v0;
        fl = r.fl;
        status = r.status;
        srad = 0.0;
        spend = spol = tronly = false;
        start = restarted = back = false;
        tr = pol = steps = tr0 = 0;
        zx = zy = -1.0;
        if (r.rst != 0) set_start(r, r.rst, g);
        return true;
    }

    // this lane's x_i, y_i from n^V: y = n^V/sum n^V, x = (z - n^V)/sum(z - n^V)
    __device__ __forceinline__ void xy_from_nv(double &x, double &y, double &bv)
    {
        const double xl = z - v0;
        const double sv = gsum<G>(v0), sl = gsum<G>(xl);
        x = xl * (1.0 / sl);
        y = v0 * (1.0 / sv);
        bv = sv;
        fl += 5 * NC + 2;
    }

    __device__ __forceinline__ void write_single(const Ctx<NC> &c, const Grp<NC, G> &g,
                                                 uint32_t bits, const int16_t (&it)[8])
    {
        const FlashArgs &a = c.a;
        if (g.act) {
            a.x[m * NC + g.gi] = z;
            a.y[m * NC + g.gi] = z;
        }
        if (g.gi == 0) {
            a.label[m] = 0;
            a.beta[m] = -1.0;
            if (a.iters) {
#pragma unroll
                for (int k = 0; k < 8; ++k) a.iters[m * 8 + k] = it[k];
            }
            if (a.status) a.status[m] = (uint16_t)bits;
            if (a.flops) a.flops[m] = fl;
        }
    }

    // Returns to the stalled split kept in the record (each lane its own
    // component): the next step evaluates it and, its trust-region budget
    // spent, reports it unconverged.
    __device__ __forceinline__ void back_to_stalled(const Ctx<NC> &c, const Grp<NC, G> &g)
    {
        v0 = g.act ? c.rec[m].lk[g.gi] : 0.0;
        back = false;
        start = spend = spol = tronly = false;
        tr0 = tr - c.a.max_tr_split;
    }

    // savef: the group's LDS holds the factor of H' at the solution.  As
    // SpNtItem::finish: false when the split restarts instead.

    __device__ __forceinline__ bool finish(const Ctx<NC> &c, const Grp<NC, G> &g, double zx_,
                                           double zy_, bool savef, double vs)
    {
        const FlashArgs &a = c.a;
        MixRec<NC> &r = c.rec[m];
        int16_t it[8];
        load_it<NC>(it, r);
        it[6] = (int16_t)tr;
        it[7] = (int16_t)pol;
        double x, y, bv;
        xy_from_nv(x, y, bv);
        const double lk = gmax<G>(g.act ? fabs(log(y / x)) : 0.0);
        const bool degenerate = !(bv > kMinPhase && bv < 1.0 - kMinPhase);
        const bool stalled = (status & kStSplitUnconv) && fmin(bv, 1.0 - bv) < kStalledPhase;
        if ((degenerate || lk < 1e-6 || stalled) && !restarted && r.wsel >= 0) {
            if (stalled && !degenerate && !(lk < 1e-6)) {
                if (g.act) r.lk[g.gi] = v0;
                back = true;
            }
            set_start(r, 1, g);
            status = (status & ~(kStSplitUnconv | kStStepCap)) | kStSplitTr | kStSplitRestart;
            return false;
        }
        if ((degenerate || lk < 1e-6) && back) {
            // the restarted descent failed: the stalled split is the result
            back_to_stalled(c, g);
            return false;
        }
        if (degenerate) {
            write_single(c, g, status | kStSplitFailed, it);
            return true;
        }
        if (lk < 1e-6) {
            write_single(c, g, status | kStSplitTrivial, it);
            return true;
        }
        const bool swap = zx_ > zy_;
        if (swap) status |= kStSwapped;
        if (g.act) {
            a.x[m * NC + g.gi] = swap ? y : x;
            a.y[m * NC + g.gi] = swap ? x : y;
            if (a.keep_factor && a.factor) {
                // factor of H~ = D^(1/2) H' D^(1/2): row i of L' scaled by 1/v_i
                const int i = g.gi;
                const double *Ls = g.lsh();
                for (int j = 0; j <= i; ++j)
                    a.factor[m * NP + i * (i + 1) / 2 + j] =
                        savef ? Ls[i * Grp<NC, G>::LD + j] / vs : NAN;
            }
        }
        if (g.gi == 0) {
            a.label[m] = 1;
            a.beta[m] = swap ? 1.0 - bv : bv;
            if (a.iters) {
#pragma unroll
                for (int k = 0; k < 8; ++k) a.iters[m * 8 + k] = it[k];
            }
            if (a.status) a.status[m] = (uint16_t)status;
            if (a.flops) a.flops[m] = fl;
        }
        return true;
    }

    __device__ __forceinline__ bool step(const Ctx<NC> &c, const Grp<NC, G> &g)
    {
        const FlashArgs &a = c.a;
        const auto kap = kappa_of<NC, PM, G>(c, m, g);
        double w0, w1, bvap;
        xy_from_nv(w0, w1, bvap);
        // scaled Hessian H' = (I - v v' + V((1-th) Phi^V + th Phi^L)V)/(th(1-th)),
        // v_i = sqrt(x_i y_i / z_i)
        const double vs = g.act ? sqrt(w0 * w1 / z) : 0.0;
        fl += 4 * NC;
        double hdiag = 0.0, dinv = 0.0;
        PhaseG o;
        phase_eval_g<NC, G>(o, g, s, b, kap, w0, fl, zx);
        zx = o.Z;
        const double th = bvap;
        phase_derivs_g<false>(hdiag, o, g, s, b, kap, th * vs, vs, fl);
        fl += 3 * NP;
        const double r0 = o.lnphi;
        const double Z0 = o.Z;
        phase_eval_g<NC, G>(o, g, s, b, kap, w1, fl, zy);
        zy = o.Z;
        phase_derivs_g<true>(hdiag, o, g, s, b, kap, (1.0 - th) * vs, vs, fl);
        // gradient of G over n^V (eq. split_grad) and G itself (eq. gibbs)
        const double fx = g.act ? log(w0) + r0 : 0.0;
        const double fy = g.act ? log(w1) + o.lnphi : 0.0;
        const double gt = fy - fx;
        const double G_ = gsum<G>((z - v0) * fx + v0 * fy);
        const double gmx = gmax<G>(fabs(gt));
        const double gs = vs * gt;
        fl += 11 * NC;
        if (start) {
            // restart: the first point whose G is below the feed's starts the
            // trust region; otherwise halve the vapour amount
            if (G_ < gf - 1e-12 * (1.0 + fabs(gf))) {
                start = false;
            } else {
                if (++nhalf > 30 || ++steps >= kStepGuard) {
                    if (back) {
                        // no start below the feed's G: the stalled split stands
                        back_to_stalled(c, g);
                        status &= ~kStSplitRestart;
                        return false;
                    }
                    int16_t it[8];
                    load_it<NC>(it, c.rec[m]);
                    it[6] = (int16_t)tr;
                    it[7] = (int16_t)pol;
                    write_single(c, g, (status & ~kStSplitRestart) | kStSplitFailed |
                                           (rstk == 2 ? kStRrNoRoot : 0u), it);
                    return true;
                }
                sb *= 0.5;
                v0 = sb * v1;
                fl += NC;
                return false;
            }
        }
        const double sc = 1.0 / (th * (1.0 - th));
        {
            double *vv = g.vec(0);
            double *hr = g.hr();
            vv[g.gi] = vs;
            wave_lds_sync();
#pragma unroll 4
            for (int j = 0; j < NC; ++j) hr[j] = g.act ? (hr[j] - vs * vv[j]) * sc : 0.0;
            wave_lds_sync();
        }
        // the identity term of H' is the diagonal addend sc
        hdiag = g.act ? (hdiag - vs * vs) * sc : 0.0;
        const double dadd = sc;
        fl += 8 * NP;
        int fin = 0;   // the split ends here: 1 without the factor, 2 with it
        do {
            if (spend) {
                spend = false;
                bool accept;
                double ratio = 1.0;
                if (fabs(spred) < 1e-13) {
                    accept = gmx < sgacc;
                } else {
                    ratio = (G_ - sfacc) / spred;
                    accept = (G_ < sfacc) && ratio > 0.0;
                }
                // a rejected or poor step halves the radius, from the length of
                // the step taken when the boundary cut made it shorter
                if (!accept) {
                    srad = 0.5 * fmin(srad, slen);
                    v0 = v1;
                    if (++steps < kStepGuard) return false;   // re-evaluate there
                    status |= kStSplitUnconv | kStStepCap;
                    fin = 1;
                    break;
                }
                if (ratio <= 0.25) srad = 0.5 * fmin(srad, slen);
                else if (ratio >= 0.75) srad *= 2.0;
            }
            if (!spol && !tronly && gmx < a.tol_split_tr) {
                spol = true;   // the paper's criterion holds: refine
                sdprev = 1e300;
            }
            // One call site for both the refinement's Newton step and the
            // trust-region step (as SpNtItem).  Newton refinement runs while H is
            // positive definite; an indefinite H sends the split back to the
            // trust region, which starts from the same point at the next step.
            const bool newton = spol;
            if (!newton) {
                if (tr - tr0 >= a.max_tr_split || ++steps >= kStepGuard) {
                    status |= kStSplitUnconv;
                    fin = 1;
                    break;
                }
                status |= kStSplitTr;
            }
            double u;
            bool eta0;
            double rad = newton ? 1e300 : srad;
            double pr = trust_step_g<NC, G>(u, rad, eta0, dinv, hdiag, dadd, gs, g, fl, newton);
            if (newton && !eta0) {
                spol = false;
                tronly = true;
                if (++steps < kStepGuard) return false;
                status |= kStSplitUnconv;
                fin = 1;
                break;
            }
            if (!newton) {
                srad = rad;
                tronly = false;
            }
            if (spol) {
                u *= vs;
                double lim = 1.0;
                if (g.act && u < 0.0) lim = fmin(lim, 0.99 * v0 / -u);
                if (g.act && u > 0.0) lim = fmin(lim, 0.99 * (z - v0) / u);
                const double dmax = gmax<G>(fabs(u));
                const double amax = gmin<G>(lim);
                v0 += amax * u;
                fl += 6 * NC;
                const bool conv = dmax < a.tol_polish || (dmax < 1e-10 && dmax >= 0.5 * sdprev);
                if (conv || pol >= a.max_polish || ++steps >= kStepGuard) {
                    if (!conv && !(dmax < 1e-10)) status |= kStSplitUnconv;
                    fin = 2;
                    break;
                }
                sdprev = dmax;
                ++pol;
                return false;
            }
            // dn = v o u, kept inside 0 < n^V < z
            const double nu = sqrt(gsum<G>(g.act ? u * u : 0.0));
            u *= vs;
            double lim = 1.0;
            if (g.act && u < 0.0) lim = fmin(lim, 0.99 * v0 / -u);
            if (g.act && u > 0.0) lim = fmin(lim, 0.99 * (z - v0) / u);
            const double amax = gmin<G>(lim);
            if (amax < 1.0) {
                const double gu = gsum<G>(gt * u);
                pr = amax * gu + amax * amax * (pr - gu);
            }
            slen = amax * nu;
            v1 = v0;
            v0 += amax * u;
            fl += 6 * NC;
            sfacc = G_;
            sgacc = gmx;
            spred = pr;
            spend = true;
            ++tr;
            return false;
        } while (false);
        return finish(c, g, Z0, o.Z, fin == 2, vs);
    }
};

}  // namespace ptf
