// flash_stages.hpp -- the flash as a pipeline of stages, each a work item
// type with begin() (cheap: load the item's state) and step() (one iteration
// of the stage; every SRK phase evaluation of the stage goes through the same
// call sites, so lanes of a wavefront evaluate the equation of state together).
//
// Stages (Sec. 2.2.3 strategy; Sec. 3 vectorisation with a barrier per stage):
//   Feed   one per mixture: feed evaluation d = ln z + ln phi(z), Wilson K,
//          the first Rachford-Rice decision (case 1 goes straight on)
//   PreSs  one per remaining mixture: the initial phase-split substitutions,
//          triage into cases 1/2/3
//   SaSs   one per stability trial (V or L): successive substitution with
//          dominant-eigenvalue acceleration (Sec. 2.2.1)
//   SaTr   one per trial that needed more: trust region in beta = 2 sqrt(W)
//          (Appendix B.1)
//   SaFin  one per analysed mixture: label decision and K re-estimate
//   SpSs   one per unstable mixture: split substitution (Sec. 2.2.2)
//   SpNt   one per split: trust region on G (Appendix B.2), Newton
//          refinement, outputs
// Items of one stage never depend on each other; a stage starts when the
// previous one has finished (kernel order on the stream).
//
// Readings of the paper used here (identical in the CPU oracle):
//   * tm carries Michelsen's leading 1 (tm = 0 at the trivial point);
//   * Delta G of the triage is (1-theta) tpd(x) + theta tpd(y);
//   * a trial is unstable when tm < -eps_tm;
//   * dominant-eigenvalue acceleration at every dem_every-th substitution
//     update u >= 2: lambda = (s_u.s_u)/(s_{u-1}.s_u), extension by
//     s_u lambda/(1 - lambda) when 0 < lambda < 1, kept only if the
//     extrapolated point lowers the objective (tm, or G per unit feed),
//     otherwise replaced by the plain update (not counted as an iteration);
//     in the split, the extrapolated point must also have a Rachford-Rice
//     root in (0,1), and no extension follows an update after which the
//     substitution stops;
//   * the trials start from the Wilson K, the initial substitutions stop at
//     the first Rachford-Rice root outside (0,1) (case 1), and a case-3 split
//     continues from the latest K with a fresh substitution budget;
//   * the split trust region is scaled: u = D^(1/2) dn with
//     D = diag(z/(x y)), the paper's shift matrix;
//   * the converged split is refined by Newton steps until max |dn| is
//     below tol_polish, and y is chosen as the phase with the larger Z;
//   * a split whose substitution leaves the two-phase region, or whose
//     first descent ends degenerate, restarts once from n^V = beta w, w the
//     composition that proved the instability (the trial the K re-estimate
//     uses, or the triage's phase with the smaller tpd), beta halved from
//     min(1, min z_i/w_i)/2 until G is below the feed's;
//   * the K re-estimate never takes a trial whose tm is not a number.
#pragma once

#include <lane_value.hpp>   // angle brackets: a host build of the items substitutes its own

#include "flash_api.hpp"
#include "srk_device.hpp"

namespace ptf {

// status bits (same values as the public header)
constexpr uint32_t kStInvalid = 0x0001u, kStShortcut = 0x0002u, kStSaRan = 0x0004u,
                   kStSaUnconv = 0x0008u, kStSplitTr = 0x0010u, kStSplitUnconv = 0x0020u,
                   kStSplitTrivial = 0x0040u, kStSplitFailed = 0x0080u,
                   kStRrNoRoot = 0x0100u, kStSwapped = 0x0200u, kStStepCap = 0x0400u,
                   kStHinted = 0x0800u, kStSplitRestart = 0x1000u;

// A split whose smaller phase holds less than this fraction of the feed is
// reported as failed (single phase).
constexpr double kMinPhase = 1e-10;

// An unconverged split whose smaller phase holds less than this fraction of
// the feed stalled against the boundary on its way to a degenerate split.
constexpr double kStalledPhase = 1e-3;

// Per-stage guard on the number of steps of one item (every stage is bounded
// by its iteration caps; this only guarantees termination).
constexpr int kStepGuard = 96;

// Per-mixture record kept in the workspace between stages.
template <int NC>
struct MixRec {
    double s[NC], b[NC];   // EOS constants at (T, P): sqrt(A_i), B_i
    double lnz[NC];        // ln of the normalised feed
    double d[NC];          // ln z + ln phi(z)
    double lkw[NC];        // initial ln K: Wilson's, or the caller's
    double lk[NC];         // split ln K (PreSs case 3, SaFin), then n^V (SpSs -> SpNt)
    double lw[2][NC];      // ln W of the stability trials (start of SaTr, final)
    double tm[2];          // final tm of the trials
    double theta;          // Rachford-Rice warm start
    uint32_t status;
    uint32_t fl;           // algorithmic flops of the mixture's sequential stages
    uint32_t tfl[2];       // flops of each trial
    uint32_t tst[2];       // status bits of each trial
    int16_t it[8];
    int32_t wsel;          // lw[wsel] holds ln of the composition that proved the
                           // instability (a trial, or the triage's phase); -1: none
    int32_t rst;           // split restart requested: 1 after theta left (0,1),
                           // 2 after a Rachford-Rice solve without root; 0: none
};


// Work lists: ids (mixture m, or trial 2m + t) and their counts.
// L_NT holds the splits that need the trust region, L_NTP those that only
// need the refinement; the last stage reads L_NT, then L_NTP, so that the
// long trust-region runs start first and the short refinements fill the end.
enum ListId : int {
    L_SA = 0, L_SATR = 1, L_SAFIN = 2, L_SPLIT = 3, L_NT = 4, L_PRE = 5, L_NTP = 6, L_COUNT = 7
};

// Device counters (list lengths, claim counters) sit 256 bytes apart: the
// atomics on them are performed where the line lives, and counters sharing
// a line would serialise each other's atomics.
constexpr int kCounterStride = 32;   // unsigned long longs

struct Lists {
    uint32_t *ids[L_COUNT];
    unsigned long long *count;   // counter block: counter k at count[k * kCounterStride]
    __host__ __device__ __forceinline__ unsigned long long *cnt(int k) const
    {
        return count + (size_t)k * kCounterStride;
    }
};

// Read-only shared component set (restrict pointers: compile-time indexed
// loads become wave-uniform scalar loads).
struct Props {
    const double *__restrict__ Tc;
    const double *__restrict__ Pc;
    const double *__restrict__ om;
    const double *__restrict__ K;
};

template <int NC>
struct Ctx {
    FlashArgs a;
    Props pr;
    MixRec<NC> *rec;
    Lists L;
};

// From this nc on, the k table of a shared set is read with vector loads
// (all lanes at the same addresses, served by the L1 cache): its nc(nc-1)/2
// values no longer fit the scalar registers, and the scalar-load form of the
// largest kernels spilled hundreds of them.
constexpr int kVectorKFromNc = 13;

// Component set of mixture m: the shared set (wave-uniform loads), or, with
// one set per mixture (PM), the mixture's own rows (nc values each, nc*nc k).
template <int NC, bool PM>
__device__ __forceinline__ Props mix_props(const Props &pr, int64_t m)
{
    if constexpr (!PM) {
        if constexpr (NC >= kVectorKFromNc) {
            return Props{pr.Tc, pr.Pc, pr.om, (const double *)per_lane((uintptr_t)pr.K)};
        } else {
            return pr;
        }
    } else {
        return Props{pr.Tc + m * NC, pr.Pc + m * NC, pr.om + m * NC, pr.K + m * NC * NC};
    }
}

// What one step of an item hands to later stages: at most two list entries,
// the first of which may be a pair of consecutive ids (the two stability
// trials 2m, 2m + 1 of a mixture).  The stage kernel appends them to the
// lists after the step, so that the appends of a wavefront can be batched.
struct Outbox {
    int l0, l1;      // list of each slot, -1 when empty
    int n0;          // ids in slot 0: 1, or 2 for a trial pair
    uint32_t i0, i1; // first id of each slot
    __device__ __forceinline__ void clear()
    {
        l0 = -1;
        l1 = -1;
        n0 = 1;
    }
    __device__ __forceinline__ void put(int list, uint32_t id)
    {
        if (l0 < 0) { l0 = list; i0 = id; n0 = 1; }
        else { l1 = list; i1 = id; }
    }
    __device__ __forceinline__ void put_pair(int list, uint32_t id)
    {
        l0 = list;
        i0 = id;
        n0 = 2;
    }
};

// ---------------------------------------------------------------------------
// Shared helpers
// ---------------------------------------------------------------------------

template <int NC>
__device__ __forceinline__ void load_z(double (&z)[NC], const FlashArgs &a, int64_t m)
{
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NC; ++i) { z[i] = a.z[m * NC + i]; s += z[i]; }
#pragma unroll
    for (int i = 0; i < NC; ++i) z[i] = z[i] / s;
}

template <int NC>
__device__ __forceinline__ void write_outputs_single(const Ctx<NC> &c, int64_t m,
                                                     const double (&z)[NC], uint32_t status,
                                                     uint32_t fl, const int16_t (&it)[8])
{
    const FlashArgs &a = c.a;
    a.label[m] = 0;
    if (a.beta) a.beta[m] = -1.0;
    if (a.x) {
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            a.x[m * NC + i] = z[i];
            a.y[m * NC + i] = z[i];
        }
    }
    if (a.iters) {
#pragma unroll
        for (int k = 0; k < 8; ++k) a.iters[m * 8 + k] = it[k];
    }
    if (a.status) a.status[m] = (uint16_t)status;
    if (a.flops) a.flops[m] = fl;
}

template <int NC>
__device__ __forceinline__ void load_it(int16_t (&it)[8], const MixRec<NC> &r)
{
#pragma unroll
    for (int k = 0; k < 8; ++k) it[k] = r.it[k];
}

// Outputs of a mixture found unstable when only the stability decision is
// asked for (no phase split): label 1 and the counters.
template <int NC>
__device__ __forceinline__ void write_outputs_unstable(const Ctx<NC> &c, int64_t m,
                                                       uint32_t status, uint32_t fl,
                                                       const int16_t (&it)[8])
{
    const FlashArgs &a = c.a;
    a.label[m] = 1;
    if (a.iters) {
#pragma unroll
        for (int k = 0; k < 8; ++k) a.iters[m * 8 + k] = it[k];
    }
    if (a.status) a.status[m] = (uint16_t)status;
    if (a.flops) a.flops[m] = fl;
}

// K -> Rachford-Rice -> normalised x, y (x_i = z_i/(1 + th(K_i - 1)),
// y_i = K_i x_i).  False when no root exists.
template <int NC>
__device__ __forceinline__ bool xy_from_lnk(double (&x)[NC], double (&y)[NC],
                                            const double (&lnk)[NC], const double (&z)[NC],
                                            double &theta, uint32_t &fl)
{
    double K[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) K[i] = exp(lnk[i]);
    fl += NC;
    if (!rr_solve<NC>(z, K, theta, fl)) return false;
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        x[i] = z[i] / (1.0 + theta * (K[i] - 1.0));
        y[i] = K[i] * x[i];
        sx += x[i];
        sy += y[i];
    }
    const double ix = 1.0 / sx, iy = 1.0 / sy;
#pragma unroll
    for (int i = 0; i < NC; ++i) { x[i] *= ix; y[i] *= iy; }
    fl += 8 * NC + 2;
    return true;
}

// One substitution update with acceleration: v += s (1 + ext); returns ext.
template <int NC>
__device__ __forceinline__ double ss_update(double (&v)[NC], double (&prev)[NC],
                                            const double (&s)[NC], int u, int dem, uint32_t &fl)
{
    double ext = 0.0;
    if (dem > 0 && u >= 2 && (u % dem) == 0) {
        double num = 0.0, den = 0.0;
#pragma unroll
        for (int i = 0; i < NC; ++i) { num += s[i] * s[i]; den += prev[i] * s[i]; }
        const double lam = num / den;
        if (lam > 0.0 && lam < 1.0) ext = lam / (1.0 - lam);
        fl += 4 * NC + 3;
    }
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        v[i] += s[i] + ext * s[i];
        prev[i] = s[i];
    }
    fl += 3 * NC;
    return ext;
}

// ---------------------------------------------------------------------------
// Feed: input checks, EOS constants, feed evaluation, Wilson K and the first
// Rachford-Rice decision of the initial substitutions (Sec. 2.2.1, 2.2.3)
// ---------------------------------------------------------------------------
template <int NC, bool PM>
__device__ __forceinline__ void wilson_lnk(double (&lk)[NC], const Props &pr, double T, double P)
{
#pragma unroll
    for (int i = 0; i < NC; ++i)
        lk[i] = log(pr.Pc[i] / P) + kWilson * (1.0 + pr.om[i]) * (1.0 - pr.Tc[i] / T);
}

// The record fields every later stage reads, and the routing of a mixture
// that leaves the initial substitutions: to the split (case 3) or to the
// stability analysis (cases 1, 2).
template <int NC>
__device__ __forceinline__ void route_mixture(MixRec<NC> &r, Outbox &ob, int64_t m, bool to_split,
                                              uint32_t status, uint32_t fl, int npre,
                                              const double (&lk)[NC], double theta)
{
#pragma unroll
    for (int i = 0; i < NC; ++i) r.lk[i] = lk[i];
    r.theta = theta;
    r.status = status;
    r.fl = fl;
    r.tfl[0] = r.tfl[1] = 0;
    r.tst[0] = r.tst[1] = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) r.it[k] = 0;
    r.it[0] = (int16_t)npre;
    r.wsel = -1;
    r.rst = 0;
    if (to_split) {
        ob.put(L_SPLIT, (uint32_t)m);
    } else {
        ob.put_pair(L_SA, (uint32_t)(2 * m));
        ob.put(L_SAFIN, (uint32_t)m);
    }
}

template <int NC, bool PM>
struct FeedItem {
    static constexpr int WAVES = 1;   // minimum wavefronts per SIMD
    static constexpr bool kPerMixture = PM;   // one component set per mixture
    static constexpr uint32_t OUT = (1u << L_SA) | (1u << L_SAFIN) | (1u << L_PRE) |
                                    (1u << L_SPLIT);   // lists the steps append to
    Outbox ob;   // list entries produced by the current step
    static constexpr int LIST = -1;   // input: mixtures 0..n-1
    static constexpr int LIST2 = -1;   // second input list, read after LIST
    int64_t m;
    double T, P;
    double z[NC];
    Eos<NC> e;

    __device__ __forceinline__ bool begin(const Ctx<NC> &c, uint32_t id)
    {
        const FlashArgs &a = c.a;
        m = id;
        const Props pp = mix_props<NC, PM>(c.pr, m);
        T = a.T[m];
        P = a.P[m];
        bool ok = (T > 0.0) && (P > 0.0) && isfinite(T) && isfinite(P);
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            const double zi = a.z[m * NC + i];
            ok = ok && (zi > 0.0) && isfinite(zi);
            z[i] = zi;
            s += zi;
        }
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            ok = ok && (pp.Tc[i] > 0.0) && (pp.Pc[i] > 0.0) && isfinite(pp.om[i]);
            ok = ok && (pp.K[i * NC + i] == 0.0);
#pragma unroll
            for (int j = 0; j < i; ++j) ok = ok && (pp.K[i * NC + j] == pp.K[j * NC + i]);
            if (a.lnk0) ok = ok && isfinite(a.lnk0[m * NC + i]);
        }
        if (!ok) {
            // invalid input: report the raw feed as a single phase
            int16_t it[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            write_outputs_single<NC>(c, m, z, kStInvalid, 0, it);
            if (c.a.tm) c.a.tm[m] = NAN;
            return false;
        }
#pragma unroll
        for (int i = 0; i < NC; ++i) z[i] = z[i] / s;
        eos_setup<NC>(e, pp.Tc, pp.Pc, pp.om, T, P);
        return true;
    }

    __device__ __forceinline__ bool step(const Ctx<NC> &c)
    {
        const FlashArgs &a = c.a;
        const int hint = a.hint ? (int)a.hint[m] : -1;
        if (hint == 0) {
            // known stable (the caller's classifier)
            int16_t it[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            write_outputs_single<NC>(c, m, z, kStHinted, 0, it);
            if (a.tm) a.tm[m] = NAN;
            return true;
        }
        const Props pp = mix_props<NC, PM>(c.pr, m);
        uint32_t fl = 0;
        Phase<NC> o;
        phase_eval<NC>(o, e, pp.K, z, fl);
        MixRec<NC> &r = c.rec[m];
        // the initial ln K: the caller's (an initializer's estimate or a
        // previous result), else Wilson's; it starts both the substitutions
        // and the two stability trials
        double ls[NC];
        if (a.lnk0) {
#pragma unroll
            for (int i = 0; i < NC; ++i) ls[i] = a.lnk0[m * NC + i];
        } else {
            wilson_lnk<NC, PM>(ls, pp, T, P);
        }
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            const double lz = log(z[i]);
            r.s[i] = e.s[i];
            r.b[i] = e.b[i];
            r.lnz[i] = lz;
            r.d[i] = lz + o.lnphi[i];
            r.lkw[i] = ls[i];
        }
        fl += 8 * NC;
        if (hint == 1) {
            // known unstable: the split starts at once
            if (a.tm) a.tm[m] = NAN;
            if (a.stability_only) {
                int16_t it[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                write_outputs_unstable<NC>(c, m, kStHinted, fl, it);
                return true;
            }
            route_mixture<NC>(r, ob, m, true, kStHinted, fl, 0, ls, 0.5);
            return true;
        }
        // the first Rachford-Rice solve of the initial substitutions decides
        // case 1 here; the other mixtures repeat it in PreSs
        double x[NC], y[NC], theta = 0.5;
        uint32_t frr = 0;
        const bool in = xy_from_lnk<NC>(x, y, ls, z, theta, frr) && theta > 0.0 && theta < 1.0;
        if (!in) {
            route_mixture<NC>(r, ob, m, false, kStSaRan, fl + frr, 0, ls, theta);
        } else {
#pragma unroll
            for (int i = 0; i < NC; ++i) r.lk[i] = ls[i];
            r.fl = fl;
            ob.put(L_PRE, (uint32_t)m);
        }
        return true;
    }
};

// ---------------------------------------------------------------------------
// PreSs: the initial phase-split substitutions and the triage (Sec. 2.2.3)
// of the mixtures that Feed did not send to case 1
// ---------------------------------------------------------------------------
template <int NC, bool PM>
struct PreSsItem {
    static constexpr int WAVES = 1;   // minimum wavefronts per SIMD
    static constexpr bool kPerMixture = PM;   // one component set per mixture
    static constexpr uint32_t OUT = (1u << L_SA) | (1u << L_SAFIN) | (1u << L_SPLIT);   // lists the steps append to
    Outbox ob;   // list entries produced by the current step
    static constexpr int LIST = L_PRE;
    static constexpr int LIST2 = -1;   // second input list, read after LIST
    int64_t m;
    double z[NC], d[NC], lk[NC];
    Eos<NC> e;
    double theta, zx, zy;   // zx, zy: Z of the previous evaluations
    int npre, steps;
    uint32_t fl;

    __device__ __forceinline__ bool begin(const Ctx<NC> &c, uint32_t id)
    {
        m = id;
        const MixRec<NC> &r = c.rec[m];
        load_z<NC>(z, c.a, m);
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            e.s[i] = r.s[i];
            e.b[i] = r.b[i];
            d[i] = r.d[i];
            lk[i] = r.lk[i];
        }
        fl = r.fl;
        theta = 0.5;
        npre = 0;
        steps = 0;
        zx = zy = -1.0;
        return true;
    }

    __device__ __forceinline__ bool step(const Ctx<NC> &c)
    {
        const Props pp = mix_props<NC, PM>(c.pr, m);
        const FlashArgs &a = c.a;
        MixRec<NC> &r = c.rec[m];
        double w0[NC], w1[NC];
        if (!(xy_from_lnk<NC>(w0, w1, lk, z, theta, fl) && theta > 0.0 && theta < 1.0)) {
            // case 1: the Rachford-Rice root left (0,1)
            route_mixture<NC>(r, ob, m, false, kStSaRan, fl, npre, lk, theta);
            return true;
        }
        Phase<NC> o;
        phase_eval<NC>(o, e, pp.K, w0, fl, zx);
        zx = o.Z;
        double r0[NC];
#pragma unroll
        for (int i = 0; i < NC; ++i) r0[i] = o.lnphi[i];
        phase_eval<NC>(o, e, pp.K, w1, fl, zy);
        zy = o.Z;
#pragma unroll
        for (int i = 0; i < NC; ++i) lk[i] = r0[i] - o.lnphi[i];
        fl += NC;
        ++npre;
        if (npre < a.max_pre_ss && ++steps < kStepGuard) return false;
        // triage (Sec. 2.2.3): tpd of the current liquid and vapour
        double tx = 0.0, ty = 0.0;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            tx += w0[i] * (log(w0[i]) + r0[i] - d[i]);
            ty += w1[i] * (log(w1[i]) + o.lnphi[i] - d[i]);
        }
        const double dg = (1.0 - theta) * tx + theta * ty;
        fl += 8 * NC + 3;
        if (tx < -a.eps_tm || ty < -a.eps_tm || dg < -a.eps_tm) {
            // case 3: unstable; the decisive value is the most negative one
            if (a.tm) a.tm[m] = fmin(tx, fmin(ty, dg));
            if (a.stability_only) {
                int16_t it[8] = {(int16_t)npre, 0, 0, 0, 0, 0, 0, 0};
                write_outputs_unstable<NC>(c, m, kStShortcut, fl, it);
                return true;
            }
            route_mixture<NC>(r, ob, m, true, kStShortcut, fl, npre, lk, 0.5);
            // the phase that proved the instability, for a restart of the split
#pragma unroll
            for (int i = 0; i < NC; ++i) r.lw[0][i] = log(tx <= ty ? w0[i] : w1[i]);
            r.wsel = 0;
        } else
            route_mixture<NC>(r, ob, m, false, kStSaRan, fl, npre, lk, theta);
        return true;
    }
};

// ---------------------------------------------------------------------------
// SaSs: successive substitution of one stability trial (Sec. 2.2.1, eq.
// ss_analyser): ln W <- d - ln phi(W)
// ---------------------------------------------------------------------------
template <int NC, bool PM>
struct SaSsItem {
    static constexpr int WAVES = 1;   // minimum wavefronts per SIMD
    static constexpr bool kPerMixture = PM;   // one component set per mixture
    static constexpr uint32_t OUT = 1u << L_SATR;   // lists the steps append to
    Outbox ob;   // list entries produced by the current step
    static constexpr int LIST = L_SA;
    static constexpr int LIST2 = -1;   // second input list, read after LIST
    int64_t m;
    int t;
    double lw[NC], prev[NC], d[NC];
    Eos<NC> e;
    double tmb, ext, zw;   // zw: Z of the previous evaluation (cubic start)
    bool dem;
    int ss, steps;
    uint32_t fl, st;

    __device__ __forceinline__ bool begin(const Ctx<NC> &c, uint32_t id)
    {
        m = id >> 1;
        t = (int)(id & 1u);
        const MixRec<NC> &r = c.rec[m];
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            e.s[i] = r.s[i];
            e.b[i] = r.b[i];
            d[i] = r.d[i];
            lw[i] = t == 0 ? r.lnz[i] + r.lkw[i] : r.lnz[i] - r.lkw[i];
        }
        fl = 2 * NC;
        st = 0;
        ss = 0;
        steps = 0;
        dem = false;
        zw = -1.0;
        return true;
    }

    __device__ __forceinline__ void done(const Ctx<NC> &c, double tm, bool to_tr)
    {
        MixRec<NC> &r = c.rec[m];
#pragma unroll
        for (int i = 0; i < NC; ++i) r.lw[t][i] = lw[i];
        r.tm[t] = tm;
        r.it[t == 0 ? 1 : 3] = (int16_t)ss;
        r.it[t == 0 ? 2 : 4] = 0;
        r.tfl[t] = fl;
        r.tst[t] = st;
        if (to_tr) ob.put(L_SATR, (uint32_t)(2 * m + t));
    }

    __device__ __forceinline__ bool step(const Ctx<NC> &c)
    {
        const Props pp = mix_props<NC, PM>(c.pr, m);
        const FlashArgs &a = c.a;
        double W[NC];
#pragma unroll
        for (int i = 0; i < NC; ++i) W[i] = exp(lw[i]);
        fl += NC;
        Phase<NC> o;
        phase_eval<NC>(o, e, pp.K, W, fl, zw);
        zw = o.Z;
        double grad[NC], tm = 1.0, gmax = 0.0;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            grad[i] = lw[i] + o.lnphi[i] - d[i];
            tm += W[i] * (grad[i] - 1.0);
            gmax = fmax(gmax, fabs(grad[i]));
        }
        fl += 6 * NC;
        if (tm < -a.eps_tm || gmax < a.tol_sa_ss) {
            done(c, tm, false);
            return true;
        }
        if (dem) {
            // an extrapolated point is kept only if it lowers tm
            dem = false;
            if (!(tm < tmb)) {
#pragma unroll
                for (int i = 0; i < NC; ++i) lw[i] -= ext * prev[i];
                if (++steps < kStepGuard) return false;
            }
        }
        if (ss < a.max_ss && ++steps < kStepGuard) {
            double s[NC];
#pragma unroll
            for (int i = 0; i < NC; ++i) s[i] = -grad[i];
            ext = ss_update<NC>(lw, prev, s, ss + 1, a.dem_every, fl);
            ++ss;
            if (ext > 0.0) {
                dem = true;
                tmb = tm;
            }
            return false;
        }
        // substitution budget spent: continue with the trust region here
        done(c, tm, true);
        return true;
    }
};

// ---------------------------------------------------------------------------
// SaTr: trust region of one trial in beta = 2 sqrt(W) (Appendix B.1,
// eqs. tr_sa, analysis_grad, analysis_hess)
// ---------------------------------------------------------------------------
template <int NC, bool PM>
struct SaTrItem {
    // two wavefronts per SIMD up to nc = 8: the item holds only ln W across
    // steps (the EOS constants, the feed reference and the last accepted point
    // stay in the record)
    static constexpr int WAVES = (NC <= 8 ? 2 : 1);   // minimum wavefronts per SIMD
    static constexpr bool kPerMixture = PM;   // one component set per mixture
    static constexpr uint32_t OUT = 0u;   // lists the steps append to
    Outbox ob;   // list entries produced by the current step
    static constexpr int LIST = L_SATR;
    static constexpr int LIST2 = -1;   // second input list, read after LIST
    static constexpr int NP = Tri<NC>::N;
    int64_t m;
    int t;
    double lw[NC];   // the current point; the record's lw[t] holds the last accepted one
    double rad, facc, pred, gacc, zw;   // zw: Z of the previous evaluation
    double slen;   // length of the last step taken, in the region's norm
    bool pend;
    int tr, steps;
    uint32_t fl, st;

    __device__ __forceinline__ bool begin(const Ctx<NC> &c, uint32_t id)
    {
        m = id >> 1;
        t = (int)(id & 1u);
        const MixRec<NC> &r = c.rec[m];
#pragma unroll
        for (int i = 0; i < NC; ++i) lw[i] = r.lw[t][i];
        fl = r.tfl[t];
        st = r.tst[t];
        rad = 0.0;
        pend = false;
        tr = 0;
        steps = 0;
        zw = -1.0;
        return true;
    }

    __device__ __forceinline__ void done(const Ctx<NC> &c, double tm)
    {
        MixRec<NC> &r = c.rec[m];
#pragma unroll
        for (int i = 0; i < NC; ++i) r.lw[t][i] = lw[i];
        r.tm[t] = tm;
        r.it[t == 0 ? 2 : 4] = (int16_t)tr;
        r.tfl[t] = fl;
        r.tst[t] = st;
    }

    __device__ __forceinline__ bool step(const Ctx<NC> &c)
    {
        const Props pp = mix_props<NC, PM>(c.pr, m);
        const FlashArgs &a = c.a;
        MixRec<NC> &r = c.rec[m];
        Eos<NC> e;
        double d[NC];
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            e.s[i] = r.s[i];
            e.b[i] = r.b[i];
            d[i] = r.d[i];
        }
        double W[NC];
#pragma unroll
        for (int i = 0; i < NC; ++i) W[i] = exp(lw[i]);
        fl += NC;
        Phase<NC> o;
        phase_eval<NC>(o, e, pp.K, W, fl, zw);
        zw = o.Z;
        double F[NP], Hs[NP], dinv[NC];
        phase_derivs<NC>(F, o, e, pp.K, fl);
        double grad[NC], g[NC], tm = 1.0, sw = 0.0, gmax = 0.0;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            grad[i] = lw[i] + o.lnphi[i] - d[i];
            tm += W[i] * (grad[i] - 1.0);
            sw += W[i];
            g[i] = sqrt(W[i]) * grad[i];
            gmax = fmax(gmax, fabs(g[i]));
        }
        fl += 9 * NC;
        if (pend) {
            pend = false;
            bool accept;
            double ratio = 1.0;
            if (fabs(pred) < 1e-13) {
                accept = gmax < gacc;
            } else {
                ratio = (tm - facc) / pred;
                accept = (tm < facc) && ratio > 0.0;
            }
            // a rejected or poor step halves the radius, from the length of
            // the step taken when the boundary cut made it shorter
            if (!accept) {
                rad = 0.5 * fmin(rad, slen);
#pragma unroll
                for (int i = 0; i < NC; ++i) lw[i] = r.lw[t][i];
                if (++steps < kStepGuard) return false;   // re-evaluate there
                st |= kStSaUnconv;
                done(c, facc);
                return true;
            }
            if (ratio <= 0.25) rad = 0.5 * fmin(rad, slen);
            else if (ratio >= 0.75) rad *= 2.0;
        }
        if (tm < -a.eps_tm || gmax < a.tol_sa_tr) {
            done(c, tm);
            return true;
        }
        if (tr >= a.max_tr_sa || ++steps >= kStepGuard) {
            st |= kStSaUnconv;
            done(c, tm);
            return true;
        }
        // H_ij = delta_ij (1 + grad_i/2) + sqrt(c_i c_j) Phi_ij
        double rc[NC];
        const double isw = 1.0 / sw;
#pragma unroll
        for (int i = 0; i < NC; ++i) rc[i] = sqrt(W[i] * isw);
#pragma unroll
        for (int i = 0; i < NC; ++i)
#pragma unroll
            for (int j = 0; j <= i; ++j)
                Hs[tri(i, j)] = rc[i] * rc[j] * F[tri(i, j)] + ((i == j) ? 1.0 + 0.5 * grad[i] : 0.0);
        fl += 2 * NP + 4 * NC;
        double u[NC];
        bool eta0;
        double pr = trust_step<NC>(u, rad, eta0, F, dinv, Hs, g, fl);
        double amax = 1.0;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            const double bi = 2.0 * sqrt(W[i]);
            if (u[i] < 0.0) amax = fmin(amax, 0.99 * bi / -u[i]);
        }
        slen = amax * norm2<NC>(u);
        if (amax < 1.0) {
            double gu = 0.0;
#pragma unroll
            for (int i = 0; i < NC; ++i) gu += g[i] * u[i];
            pr = amax * gu + amax * amax * (pr - gu);
        }
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            r.lw[t][i] = lw[i];
            lw[i] = 2.0 * log(sqrt(W[i]) + 0.5 * amax * u[i]);
        }
        fl += 6 * NC;
        facc = tm;
        gacc = gmax;
        pred = pr;
        pend = true;
        ++tr;
        return false;
    }
};

// ---------------------------------------------------------------------------
// SaFin: label decision and K re-estimate (Sec. 2.2.1, last paragraph)
// ---------------------------------------------------------------------------
template <int NC, bool PM>
struct SaFinItem {
    static constexpr int WAVES = 1;   // minimum wavefronts per SIMD
    static constexpr bool kPerMixture = PM;   // one component set per mixture
    static constexpr uint32_t OUT = 1u << L_SPLIT;   // lists the steps append to
    Outbox ob;   // list entries produced by the current step
    static constexpr int LIST = L_SAFIN;
    static constexpr int LIST2 = -1;   // second input list, read after LIST
    int64_t m;

    __device__ __forceinline__ bool begin(const Ctx<NC> &c, uint32_t id)
    {
        m = id;
        return true;
    }

    __device__ __forceinline__ bool step(const Ctx<NC> &c)
    {
        MixRec<NC> &r = c.rec[m];
        const double t0 = r.tm[0], t1 = r.tm[1];
        const uint32_t status = r.status | r.tst[0] | r.tst[1];
        uint32_t fl = r.fl + r.tfl[0] + r.tfl[1];
        const bool unstable = (t0 < -c.a.eps_tm) || (t1 < -c.a.eps_tm);
        if (c.a.tm) c.a.tm[m] = fmin(t0, t1);
        if (unstable && c.a.stability_only) {
            int16_t it[8];
            load_it<NC>(it, r);
            write_outputs_unstable<NC>(c, m, status, fl, it);
            return true;
        }
        if (!unstable) {
            double z[NC];
            load_z<NC>(z, c.a, m);
            int16_t it[8];
            load_it<NC>(it, r);
            write_outputs_single<NC>(c, m, z, status, fl, it);
            return true;
        }
        // the trial with the smaller tm; a trial whose substitution diverged
        // (tm not a number) is never the one taken
        const int ts = (t1 < t0 || isnan(t0)) ? 1 : 0;
        if (ts == 1) {
#pragma unroll
            for (int i = 0; i < NC; ++i) r.lk[i] = r.lnz[i] - r.lw[1][i];
        } else {
#pragma unroll
            for (int i = 0; i < NC; ++i) r.lk[i] = r.lw[0][i] - r.lnz[i];
        }
        r.wsel = ts;
        r.theta = 0.5;
        r.status = status;
        r.fl = fl + NC;
        ob.put(L_SPLIT, (uint32_t)m);
        return true;
    }
};

// ---------------------------------------------------------------------------
// SpSs: successive substitution of the split (Sec. 2.2.2)
// ---------------------------------------------------------------------------
template <int NC, bool PM>
struct SpSsItem {
    static constexpr int WAVES = (NC <= 8 ? 2 : 1);   // minimum wavefronts per SIMD
    static constexpr bool kPerMixture = PM;   // one component set per mixture
    static constexpr uint32_t OUT = (1u << L_NT) | (1u << L_NTP);   // lists the steps append to
    Outbox ob;   // list entries produced by the current step
    static constexpr int LIST = L_SPLIT;
    static constexpr int LIST2 = -1;   // second input list, read after LIST
    int64_t m;
    double z[NC], lk[NC], prev[NC];
    Eos<NC> e;
    double theta, sgb, sext, zx, zy;   // zx, zy: Z of the previous evaluations
    bool dem;
    int ss, steps;
    uint32_t fl, status;

    __device__ __forceinline__ bool begin(const Ctx<NC> &c, uint32_t id)
    {
        m = id;
        const MixRec<NC> &r = c.rec[m];
        load_z<NC>(z, c.a, m);
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            e.s[i] = r.s[i];
            e.b[i] = r.b[i];
            lk[i] = r.lk[i];
        }
        theta = r.theta;
        fl = r.fl;
        status = r.status;
        ss = 0;
        steps = 0;
        dem = false;
        zx = zy = -1.0;
        return true;
    }

    __device__ __forceinline__ void fail(const Ctx<NC> &c, uint32_t bits)
    {
        MixRec<NC> &r = c.rec[m];
        int16_t it[8];
        load_it<NC>(it, r);
        it[5] = (int16_t)ss;
        write_outputs_single<NC>(c, m, z, status | bits, fl, it);
    }

    // The substitution left the two-phase region (no Rachford-Rice root, or
    // theta outside (0,1)): the split restarts in the trust-region stage from
    // the composition that proved the instability, when there is one;
    // otherwise the mixture is reported single phase (SPLIT_FAILED).
    __device__ __forceinline__ void restart_or_fail(const Ctx<NC> &c, bool no_root,
                                                    uint32_t fail_bits)
    {
        MixRec<NC> &r = c.rec[m];
        if (r.wsel < 0) {
            fail(c, kStSplitFailed | (no_root ? kStRrNoRoot : 0u) | fail_bits);
            return;
        }
        r.rst = no_root ? 2 : 1;
        r.it[5] = (int16_t)ss;
        r.fl = fl;
        r.status = status | kStSplitTr | kStSplitRestart;
        ob.put(L_NT, (uint32_t)m);
    }

    __device__ __forceinline__ bool step(const Ctx<NC> &c)
    {
        const Props pp = mix_props<NC, PM>(c.pr, m);
        const FlashArgs &a = c.a;
        double x[NC], y[NC];
        if (!xy_from_lnk<NC>(x, y, lk, z, theta, fl)) {
            if (dem) {
                // an extrapolated point without a Rachford-Rice root is
                // rejected like one that does not lower G
                dem = false;
#pragma unroll
                for (int i = 0; i < NC; ++i) lk[i] -= sext * prev[i];
                if (++steps < kStepGuard) return false;
            }
            restart_or_fail(c, true, 0u);
            return true;
        }
        Phase<NC> o;
        phase_eval<NC>(o, e, pp.K, x, fl, zx);
        zx = o.Z;
        double r0[NC];
#pragma unroll
        for (int i = 0; i < NC; ++i) r0[i] = o.lnphi[i];
        phase_eval<NC>(o, e, pp.K, y, fl, zy);
        zy = o.Z;
        // G per unit feed (eq. gibbs) where an acceleration check needs it
        const bool dem_next = a.dem_every > 0 && ss + 1 >= 2 && ((ss + 1) % a.dem_every) == 0;
        double G = 0.0;
        if (dem || dem_next) {
#pragma unroll
            for (int i = 0; i < NC; ++i)
                G += (1.0 - theta) * x[i] * (log(x[i]) + r0[i]) + theta * y[i] * (log(y[i]) + o.lnphi[i]);
            fl += 10 * NC;
        }
        if (dem) {
            // an extrapolated point is kept only if it is a physical split
            // (0 < theta < 1, where G is the Gibbs energy of two phases) and
            // lowers G
            dem = false;
            if (!(theta > 0.0 && theta < 1.0 && G < sgb)) {
#pragma unroll
                for (int i = 0; i < NC; ++i) lk[i] -= sext * prev[i];
                if (++steps < kStepGuard) return false;
            }
        }
        double s[NC], dmax = 0.0;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            s[i] = (r0[i] - o.lnphi[i]) - lk[i];
            dmax = fmax(dmax, fabs(exp(s[i]) - 1.0));
        }
        fl += 4 * NC;
        // no extension on an update after which the substitution stops: no
        // later evaluation could check the extrapolated point
        const bool conv = dmax < a.tol_split_ss;
        const bool more = !conv && ss + 1 < a.max_ss && steps + 1 < kStepGuard;
        const double ext = ss_update<NC>(lk, prev, s, ss + 1, more ? a.dem_every : 0, fl);
        ++ss;
        if (more) {
            ++steps;
            if (ext > 0.0) {
                dem = true;
                sgb = G;
                sext = ext;
            }
            return false;
        }
        // hand over to the trust region: n^V = theta y from the final K
        MixRec<NC> &r = c.rec[m];
        if (!xy_from_lnk<NC>(x, y, lk, z, theta, fl)) {
            restart_or_fail(c, true, conv ? 0u : kStSplitTr);
            return true;
        }
        if (!(theta > 0.0 && theta < 1.0)) {
            restart_or_fail(c, false, conv ? 0u : kStSplitTr);
            return true;
        }
#pragma unroll
        for (int i = 0; i < NC; ++i) r.lk[i] = theta * y[i];
        r.it[5] = (int16_t)ss;
        r.fl = fl;
        r.status = status | (conv ? 0u : kStSplitTr);
        ob.put(conv ? L_NTP : L_NT, (uint32_t)m);
        return true;
    }
};

// ---------------------------------------------------------------------------
// SpNt: trust region on G over n^V (Appendix B.2, eqs. newton_splitter,
// split_grad, split_hess), Newton refinement, outputs
// ---------------------------------------------------------------------------
template <int NC, bool PM>
struct SpNtItem {
    static constexpr int WAVES = 1;   // minimum wavefronts per SIMD
    static constexpr bool kPerMixture = PM;   // one component set per mixture
    static constexpr uint32_t OUT = 0u;   // lists the steps append to
    Outbox ob;   // list entries produced by the current step
    static constexpr int LIST = L_NT;
    static constexpr int LIST2 = L_NTP;   // refinement-only splits, read after L_NT
    static constexpr int NP = Tri<NC>::N;
    int64_t m;
    double z[NC], v0[NC], v1[NC];
    Eos<NC> e;
    double srad, sfacc, spred, sgacc, sdprev, zx, zy;   // zx, zy: previous Z
    double slen;   // scaled length of the last trust-region step taken
    double sb, gf; // restart: current vapour amount of the start search, feed G
    bool spend, spol;
    bool tronly;   // refinement found H indefinite: take a trust-region step first
    bool start;    // restart: searching the start point (v1 holds the composition)
    bool restarted;
    bool back;     // the record holds a stalled first descent's point (r.lk)
    int tr, pol, steps, nhalf, rstk;
    int tr0;       // trust-region steps before a restart (each descent has the cap)
    uint32_t fl, status;

    // Restart of the split from the composition w that proved the
    // instability (record field lw[wsel]): n^V = beta w with
    // beta = min(1, min_i z_i / w_i) / 2, halved until G is below the
    // feed's (in step).  rs: the record's restart code.
    __device__ __forceinline__ void set_start(const MixRec<NC> &r, int rs)
    {
        double sw = 0.0, bmax = 1.0, g = 0.0;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            v1[i] = exp(r.lw[r.wsel][i]);
            sw += v1[i];
        }
        const double isw = 1.0 / sw;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            v1[i] *= isw;
            bmax = fmin(bmax, z[i] / v1[i]);
            g += z[i] * r.d[i];
        }
        sb = 0.5 * bmax;
#pragma unroll
        for (int i = 0; i < NC; ++i) v0[i] = sb * v1[i];
        gf = g;
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

    __device__ __forceinline__ bool begin(const Ctx<NC> &c, uint32_t id)
    {
        m = id;
        const MixRec<NC> &r = c.rec[m];
        load_z<NC>(z, c.a, m);
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            e.s[i] = r.s[i];
            e.b[i] = r.b[i];
            v0[i] = r.lk[i];
        }
        fl = r.fl;
        status = r.status;
        srad = 0.0;
        spend = spol = tronly = false;
        start = restarted = back = false;
        tr = pol = steps = tr0 = 0;
        zx = zy = -1.0;
        if (r.rst != 0) set_start(r, r.rst);
        return true;
    }

    // Returns to the stalled split kept in the record: the next step
    // evaluates it and, its trust-region budget spent, reports it
    // unconverged.
    __device__ __forceinline__ void back_to_stalled(const Ctx<NC> &c)
    {
        const MixRec<NC> &r = c.rec[m];
#pragma unroll
        for (int i = 0; i < NC; ++i) v0[i] = r.lk[i];
        back = false;
        start = spend = spol = tronly = false;
        tr0 = tr - c.a.max_tr_split;
    }

    // x, y from v0 = n^V: y = n^V/sum n^V, x = (z - n^V)/sum(z - n^V)
    __device__ __forceinline__ void xy_from_nv(double (&x)[NC], double (&y)[NC], double &bv)
    {
        double sv = 0.0, sl = 0.0;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            x[i] = z[i] - v0[i];
            y[i] = v0[i];
            sv += y[i];
            sl += x[i];
        }
        const double iv = 1.0 / sv, il = 1.0 / sl;
#pragma unroll
        for (int i = 0; i < NC; ++i) { x[i] *= il; y[i] *= iv; }
        bv = sv;
        fl += 5 * NC + 2;
    }

    // Writes the outputs and returns true, or, when the split ended
    // degenerate (a phase below kMinPhase of the feed), at the trivial point
    // (no unstable feed's split: the composition that proved the instability
    // gives a lower G) or unconverged with a phase below kStalledPhase, and
    // has not been restarted yet, restarts it from that composition and
    // returns false.  A stalled split is kept in the record (n^V in lk,
    // unused from here on) and is the result, flagged unconverged, when the
    // restarted descent ends degenerate or trivial.
    __device__ __forceinline__ bool finish(const Ctx<NC> &c, double zx, double zy,
                                           const double (&Lf)[NP], bool savef,
                                           const double (&vs)[NC])
    {
        const FlashArgs &a = c.a;
        MixRec<NC> &r = c.rec[m];
        int16_t it[8];
        load_it<NC>(it, r);
        it[6] = (int16_t)tr;
        it[7] = (int16_t)pol;
        double x[NC], y[NC], bv;
        xy_from_nv(x, y, bv);
        double lk = 0.0;
#pragma unroll
        for (int i = 0; i < NC; ++i) lk = fmax(lk, fabs(log(y[i] / x[i])));
        const bool degenerate = !(bv > kMinPhase && bv < 1.0 - kMinPhase);
        const bool stalled = (status & kStSplitUnconv) && fmin(bv, 1.0 - bv) < kStalledPhase;
        if ((degenerate || lk < 1e-6 || stalled) && !restarted && r.wsel >= 0) {
            if (stalled && !degenerate && !(lk < 1e-6)) {
#pragma unroll
                for (int i = 0; i < NC; ++i) r.lk[i] = v0[i];
                back = true;
            }
            set_start(r, 1);
            status = (status & ~(kStSplitUnconv | kStStepCap)) | kStSplitTr | kStSplitRestart;
            return false;
        }
        if ((degenerate || lk < 1e-6) && back) {
            // the restarted descent failed: the stalled split is the result
            back_to_stalled(c);
            return false;
        }
        if (degenerate) {
            write_outputs_single<NC>(c, m, z, status | kStSplitFailed, fl, it);
            return true;
        }
        if (lk < 1e-6) {
            write_outputs_single<NC>(c, m, z, status | kStSplitTrivial, fl, it);
            return true;
        }
        const bool swap = zx > zy;
        if (swap) status |= kStSwapped;
        a.label[m] = 1;
        a.beta[m] = swap ? 1.0 - bv : bv;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            a.x[m * NC + i] = swap ? y[i] : x[i];
            a.y[m * NC + i] = swap ? x[i] : y[i];
        }
        if (a.keep_factor && a.factor) {
            // factor of H~ = D^(1/2) H' D^(1/2): row i of L' scaled by 1/v_i
#pragma unroll
            for (int i = 0; i < NC; ++i)
#pragma unroll
                for (int j = 0; j <= i; ++j)
                    a.factor[m * NP + tri(i, j)] = savef ? Lf[tri(i, j)] / vs[i] : NAN;
        }
        if (a.iters) {
#pragma unroll
            for (int k = 0; k < 8; ++k) a.iters[m * 8 + k] = it[k];
        }
        if (a.status) a.status[m] = (uint16_t)status;
        if (a.flops) a.flops[m] = fl;
        return true;
    }

    __device__ __forceinline__ bool step(const Ctx<NC> &c)
    {
        const Props pp = mix_props<NC, PM>(c.pr, m);
        const FlashArgs &a = c.a;
        double w0[NC], w1[NC], bvap;
        xy_from_nv(w0, w1, bvap);
        // scaled Hessian H' = (I - v v' + V((1-th) Phi^V + th Phi^L)V)/(th(1-th)),
        // v_i = sqrt(x_i y_i / z_i), accumulated over the two evaluations
        double vs[NC];
#pragma unroll
        for (int i = 0; i < NC; ++i) vs[i] = sqrt(w0[i] * w1[i] / z[i]);
        fl += 4 * NC;
        double F[NP], Hs[NP], dinv[NC];
        Phase<NC> o;
        phase_eval<NC>(o, e, pp.K, w0, fl, zx);
        zx = o.Z;
        phase_derivs<NC>(F, o, e, pp.K, fl);
#pragma unroll
        for (int i = 0; i < NC; ++i)
#pragma unroll
            for (int j = 0; j <= i; ++j) Hs[tri(i, j)] = bvap * vs[i] * vs[j] * F[tri(i, j)];
        fl += 3 * NP;
        double r0[NC];
        const double Z0 = o.Z;
#pragma unroll
        for (int i = 0; i < NC; ++i) r0[i] = o.lnphi[i];
        phase_eval<NC>(o, e, pp.K, w1, fl, zy);
        zy = o.Z;
        phase_derivs<NC>(F, o, e, pp.K, fl);
        const double th = bvap;
        // gradient of G over n^V (eq. split_grad) and G itself (eq. gibbs)
        double gt[NC], gs[NC], G = 0.0, gmax = 0.0;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            const double fx = log(w0[i]) + r0[i];
            const double fy = log(w1[i]) + o.lnphi[i];
            gt[i] = fy - fx;
            G += (z[i] - v0[i]) * fx + v0[i] * fy;
            gmax = fmax(gmax, fabs(gt[i]));
            gs[i] = vs[i] * gt[i];
        }
        fl += 11 * NC;
        if (start) {
            // restart: the first point whose G is below the feed's starts the
            // trust region; otherwise halve the vapour amount
            if (G < gf - 1e-12 * (1.0 + fabs(gf))) {
                start = false;
            } else {
                if (++nhalf > 30 || ++steps >= kStepGuard) {
                    if (back) {
                        // no start below the feed's G: the stalled split stands
                        back_to_stalled(c);
                        status &= ~kStSplitRestart;
                        return false;
                    }
                    int16_t it[8];
                    load_it<NC>(it, c.rec[m]);
                    it[6] = (int16_t)tr;
                    it[7] = (int16_t)pol;
                    write_outputs_single<NC>(
                        c, m, z, (status & ~kStSplitRestart) | kStSplitFailed |
                                     (rstk == 2 ? kStRrNoRoot : 0u), fl, it);
                    return true;
                }
                sb *= 0.5;
#pragma unroll
                for (int i = 0; i < NC; ++i) v0[i] = sb * v1[i];
                fl += NC;
                return false;
            }
        }
        const double sc = 1.0 / (th * (1.0 - th));
#pragma unroll
        for (int i = 0; i < NC; ++i)
#pragma unroll
            for (int j = 0; j <= i; ++j) {
                double h = Hs[tri(i, j)] + (1.0 - th) * vs[i] * vs[j] * F[tri(i, j)] - vs[i] * vs[j];
                if (i == j) h += 1.0;
                Hs[tri(i, j)] = h * sc;
            }
        fl += 8 * NP;
        int fin = 0;   // the split ends here: 1 without the factor, 2 with it
        do {
            if (spend) {
                spend = false;
                bool accept;
                double ratio = 1.0;
                if (fabs(spred) < 1e-13) {
                    accept = gmax < sgacc;
                } else {
                    ratio = (G - sfacc) / spred;
                    accept = (G < sfacc) && ratio > 0.0;
                }
                // a rejected or poor step halves the radius, from the length of
                // the step taken when the boundary cut made it shorter
                if (!accept) {
                    srad = 0.5 * fmin(srad, slen);
    #pragma unroll
                    for (int i = 0; i < NC; ++i) v0[i] = v1[i];
                    if (++steps < kStepGuard) return false;   // re-evaluate there
                    status |= kStSplitUnconv | kStStepCap;
                    fin = 1;
                    break;
                }
                if (ratio <= 0.25) srad = 0.5 * fmin(srad, slen);
                else if (ratio >= 0.75) srad *= 2.0;
            }
            if (!spol && !tronly && gmax < a.tol_split_tr) {
                spol = true;   // the paper's criterion holds: refine
                sdprev = 1e300;
            }
            // One call site for both the refinement's Newton step and the
            // trust-region step, so that lanes in either mode factor together.
            // Newton refinement runs while H is positive definite; an indefinite
            // H sends the split back to the trust region, which starts from the
            // same point at the next step.
            const bool newton = spol;
            if (!newton) {
                if (tr - tr0 >= a.max_tr_split || ++steps >= kStepGuard) {
                    status |= kStSplitUnconv;
                    fin = 1;
                    break;
                }
                status |= kStSplitTr;
            }
            double u[NC];
            bool eta0;
            double rad = newton ? 1e300 : srad;
            double pr = trust_step<NC>(u, rad, eta0, F, dinv, Hs, gs, fl, newton);
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
                double dmax = 0.0, amax = 1.0;
    #pragma unroll
                for (int i = 0; i < NC; ++i) {
                    u[i] *= vs[i];
                    dmax = fmax(dmax, fabs(u[i]));
                    if (u[i] < 0.0) amax = fmin(amax, 0.99 * v0[i] / -u[i]);
                    if (u[i] > 0.0) amax = fmin(amax, 0.99 * (z[i] - v0[i]) / u[i]);
                }
    #pragma unroll
                for (int i = 0; i < NC; ++i) v0[i] += amax * u[i];
                fl += 6 * NC;
                // converged: step below tol_polish, or rounding-size steps that no
                // longer shrink
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
            const double nu = norm2<NC>(u);
            double amax = 1.0;
    #pragma unroll
            for (int i = 0; i < NC; ++i) {
                u[i] *= vs[i];
                if (u[i] < 0.0) amax = fmin(amax, 0.99 * v0[i] / -u[i]);
                if (u[i] > 0.0) amax = fmin(amax, 0.99 * (z[i] - v0[i]) / u[i]);
            }
            if (amax < 1.0) {
                double gu = 0.0;
    #pragma unroll
                for (int i = 0; i < NC; ++i) gu += gt[i] * u[i];
                pr = amax * gu + amax * amax * (pr - gu);
            }
            slen = amax * nu;
    #pragma unroll
            for (int i = 0; i < NC; ++i) {
                v1[i] = v0[i];
                v0[i] += amax * u[i];
            }
            fl += 6 * NC;
            sfacc = G;
            sgacc = gmax;
            spred = pr;
            spend = true;
            ++tr;
            return false;
        } while (false);
        return finish(c, Z0, o.Z, F, fin == 2, vs);
    }
};

}  // namespace ptf
