// flash_launch.hpp -- kernels of the flash and their host-side launchers for
// one component count.  Included only by flash_nc.hip, which is compiled
// once per nc and instantiates the nc_* entry points declared in
// flash_api.hpp; everything else here has internal linkage.
//
// The flash runs as a pipeline of stage kernels (flash_stages.hpp): every
// stage is a persistent grid whose wavefronts take work items (mixtures or
// stability trials) from a device list, one item per lane, and refill a lane
// as soon as its item finishes; an item that needs a later stage is appended
// to that stage's list.  This is the paper's synchronizer (save converged
// rows, drop them from the active set) and its barrier per stage (Sec. 3,
// Algorithm 1), done on the device without host synchronisation: the kernel
// order on the stream is the barrier.  The plain form runs the same items
// one step per launch, with compaction and a host read of the active count
// after every launch.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "flash_api.hpp"
#include "flash_stages.hpp"
#include "flash_group.hpp"
#include "adjoint_device.hpp"
#include "tuned_gfx950.hpp"

namespace ptf {
namespace {

constexpr int kBlock = 256;

// Zeroes n counters of a counter block (kCounterStride apart).
__global__ void reset_counters(unsigned long long *q, int n)
{
    if ((int)threadIdx.x < n) q[(size_t)threadIdx.x * kCounterStride] = 0ull;
}

// Number of items of a stage: all mixtures for the first stage, else the
// length of the stage's list (written by the previous stages).
template <class Item, int NC>
__device__ __forceinline__ int64_t stage_count(const Ctx<NC> &c)
{
    if (Item::LIST < 0) return c.a.n;
    int64_t k = (int64_t)*c.L.cnt(Item::LIST);
    if (Item::LIST2 >= 0) k += (int64_t)*c.L.cnt(Item::LIST2 < 0 ? 0 : Item::LIST2);
    return k;
}

// Id of input entry k: entries of LIST first, then those of LIST2.
template <class Item, int NC>
__device__ __forceinline__ uint32_t stage_id(const Ctx<NC> &c, int64_t k)
{
    if (Item::LIST < 0) return (uint32_t)k;
    constexpr int l1 = Item::LIST < 0 ? 0 : Item::LIST;
    if (Item::LIST2 >= 0) {
        constexpr int l2 = Item::LIST2 < 0 ? 0 : Item::LIST2;
        const int64_t n1 = (int64_t)*c.L.cnt(l1);
        if (k >= n1) return c.L.ids[l2][k - n1];
    }
    return c.L.ids[l1][k];
}

// Ids a wavefront claims from a stage's input with one atomic (after its
// static first share, three quarters of an even split of the input).
constexpr int kChunk = 64;
// Per-wavefront staging of list appends in LDS (entries per output list).
constexpr int kStage = 512;
constexpr int kWavesPerBlock = kBlock / 64;

// Output lists of a stage: bit l of Item::OUT; slot_of<OUT>(l) is the list's
// staging buffer.
__host__ __device__ constexpr int popcount32(uint32_t v)
{
    return v == 0u ? 0 : (int)(v & 1u) + popcount32(v >> 1);
}
template <uint32_t OUT>
__device__ constexpr int slot_of(int l)
{
    return popcount32(OUT & ((1u << l) - 1u));
}

// Wave-level helpers (called by all 64 lanes together).
__device__ __forceinline__ unsigned long long lanes_below(int lane)
{
    return (1ull << lane) - 1ull;
}

__device__ __forceinline__ unsigned long long bcast64(unsigned long long v, int src)
{
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, src);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), src);
    return ((unsigned long long)hi << 32) | lo;
}

// Input positions a wavefront takes from its stage's input.  First its
// static share, a contiguous range of three quarters of the input split
// evenly (consecutive lanes take consecutive positions, which keeps the
// mixtures a wavefront touches, and the records it reads, close together in
// memory); then chunks of kChunk positions from the stage's counter, one
// atomic per chunk.
struct Claim {
    unsigned long long nw, wid, s0, sj, dyn0, cb, ce;   // [cb, ce): claimed, not yet taken

    __device__ __forceinline__ Claim(int64_t count, unsigned long long nw_,
                                     unsigned long long wid_)
        : nw(nw_), wid(wid_), sj(0), cb(0), ce(0)
    {
        s0 = (unsigned long long)(count > 0 ? count : 0) * 3ull / 4ull / nw;
        dyn0 = nw * s0;
    }

    // Called by every lane of the wavefront with the number r (1..64) of
    // takers; returns the position for the taker of rank `rank` (used in
    // the taker lanes only).
    __device__ __forceinline__ unsigned long long next(int r, unsigned long long rank, int lane,
                                                       unsigned long long *take)
    {
        const unsigned long long ru = (unsigned long long)r;
        const unsigned long long as = s0 - sj, ad = ce - cb;
        unsigned long long nb = 0;
        if (as + ad < ru) {
            if (lane == 0) nb = dyn0 + atomicAdd(take, (unsigned long long)kChunk);
            nb = bcast64(nb, 0);
        }
        unsigned long long k;
        if (rank < as) k = wid * s0 + sj + rank;
        else if (rank - as < ad) k = cb + (rank - as);
        else k = nb + (rank - as - ad);
        if (ru <= as) {
            sj += ru;
        } else {
            sj = s0;
            const unsigned long long rem = ru - as;
            if (rem <= ad) {
                cb += rem;
            } else {
                cb = nb + (rem - ad);
                ce = nb + kChunk;
            }
        }
        return k;
    }
};

// Copies a wavefront's staged entries of one list to the global list: one
// atomic for the whole batch, then a coalesced copy.
__device__ __forceinline__ void flush_list(const Lists &L, int list, const uint32_t *buf,
                                           int fill, int lane)
{
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(L.cnt(list), (unsigned long long)fill);
    base = bcast64(base, 0);
    for (int k = lane; k < fill; k += 64) L.ids[list][base + (unsigned long long)k] = buf[k];
}

// Stages the entries of one outbox slot (list l, first id i, n ids) of every
// lane whose slot names `list`.
__device__ __forceinline__ void stage_slot(const Lists &L, int list, int l, uint32_t i, int n,
                                           uint32_t *buf, int &fill, int lane)
{
    const bool mine = (l == list);
    const unsigned long long m1 = __ballot(mine);
    if (m1 == 0ull) return;
    const unsigned long long m2 = __ballot(mine && n == 2);
    const int tot = __popcll(m1) + __popcll(m2);
    if (fill + tot > kStage) {
        flush_list(L, list, buf, fill, lane);
        fill = 0;
    }
    if (mine) {
        const unsigned long long b = lanes_below(lane);
        const int r = fill + __popcll(m1 & b) + __popcll(m2 & b);
        buf[r] = i;
        if (n == 2) buf[r + 1] = i + 1u;
    }
    fill += tot;
}

// Appends the entries of one outbox slot of every active lane whose slot
// names `list` directly to the global list (one atomic per wavefront; the
// plain form, where lanes beyond the active count have returned).
__device__ __forceinline__ void append_slot(const Lists &L, int list, int l, uint32_t i, int n,
                                            int lane)
{
    const bool mine = (l == list);
    const unsigned long long m1 = __ballot(mine);
    if (m1 == 0ull) return;
    const unsigned long long m2 = __ballot(mine && n == 2);
    const int tot = __popcll(m1) + __popcll(m2);
    const int leader = __ffsll((unsigned long long)__ballot(1)) - 1;   // lowest active lane
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(L.cnt(list), (unsigned long long)tot);
    base = bcast64(base, leader);
    if (mine) {
        const unsigned long long b = lanes_below(lane);
        const unsigned long long r = base + (unsigned long long)(__popcll(m1 & b) + __popcll(m2 & b));
        L.ids[list][r] = i;
        if (n == 2) L.ids[list][r + 1] = i + 1u;
    }
}

// Persistent stage: one item per lane; lanes whose item finished take the
// next input positions of the wavefront (Claim: a static share, then
// chunks of kChunk from the stage's counter).  The
// list entries the steps produce are staged per wavefront in LDS and
// appended kStage at a time (one atomic per batch).  Every item finishes
// within its stage's iteration caps (and kStepGuard steps), so every
// wavefront reaches the exit, where it appends what it still holds.
template <class Item, int NC>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(Item::WAVES)))
stage_persistent(Ctx<NC> c, const double *__restrict__ Tc, const double *__restrict__ Pc,
                 const double *__restrict__ om, const double *__restrict__ K,
                 unsigned long long *__restrict__ take)
{
    constexpr uint32_t OUT = Item::OUT;
    constexpr int NOUT = popcount32(OUT) > 0 ? popcount32(OUT) : 1;
    __shared__ uint32_t stage_buf[kWavesPerBlock][NOUT][kStage];
    c.pr = Props{Tc, Pc, om, K};
    const int64_t count = stage_count<Item, NC>(c);
    const int lane = (int)__lane_id();
    uint32_t(*buf)[kStage] = stage_buf[threadIdx.x / 64];
    int fill[NOUT];
#pragma unroll
    for (int l = 0; l < NOUT; ++l) fill[l] = 0;
    Claim cl(count, (unsigned long long)gridDim.x * (blockDim.x / 64),
             (unsigned long long)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64);
    Item it;
    bool live = false, gone = false;
    for (;;) {
        const bool want = !live && !gone;
        const unsigned long long mask = __ballot(want);
        if (mask) {
            const unsigned long long rank = (unsigned long long)__popcll(mask & lanes_below(lane));
            const unsigned long long k = cl.next(__popcll(mask), rank, lane, take);
            if (want) {
                if ((int64_t)k < count) live = it.begin(c, stage_id<Item, NC>(c, (int64_t)k));
                else gone = true;
            }
        }
        if (__ballot(!gone) == 0ull) break;
        it.ob.clear();
        if (live) live = !it.step(c);
#pragma unroll
        for (int l = 0; l < L_COUNT; ++l) {
            if ((OUT >> l) & 1u) {
                const int q = slot_of<OUT>(l);
                stage_slot(c.L, l, it.ob.l0, it.ob.i0, it.ob.n0, buf[q], fill[q], lane);
                stage_slot(c.L, l, it.ob.l1, it.ob.i1, 1, buf[q], fill[q], lane);
            }
        }
    }
#pragma unroll
    for (int l = 0; l < L_COUNT; ++l) {
        if ((OUT >> l) & 1u) {
            const int q = slot_of<OUT>(l);
            if (fill[q] > 0) flush_list(c.L, l, buf[q], fill[q], lane);
        }
    }
}

// Persistent stage with one group of G lanes per item (flash_group.hpp): as
// stage_persistent, with groups in place of lanes.  The lowest lane of each
// group takes part in the claim and holds the group's list entries.
template <class Item, int NC, int G>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(Item::WAVES)))
stage_persistent_group(Ctx<NC> c, const double *__restrict__ Tc, const double *__restrict__ Pc,
                       const double *__restrict__ om, const double *__restrict__ K,
                       unsigned long long *__restrict__ take)
{
    static_assert(64 % G == 0 && G >= NC, "a group spans the components within one wavefront");
    constexpr uint32_t OUT = Item::OUT;
    constexpr int NOUT = popcount32(OUT) > 0 ? popcount32(OUT) : 1;
    __shared__ uint32_t stage_buf[kWavesPerBlock][NOUT][kStage];
    // dynamic LDS (group_lds_bytes): for a shared component set the table
    // kappa_ij = 1 - k_ij, once per block with rows KapLds::stride<NC>()
    // apart, then the region of each group of the block
    extern __shared__ double group_dyn[];
    constexpr int KS = KapLds::stride<NC>();
    constexpr int KN = Item::kPerMixture ? 0 : NC * KS;
    double *kap_lds = group_dyn;
    c.pr = Props{Tc, Pc, om, K};
    if constexpr (!Item::kPerMixture) {
        for (int t = (int)threadIdx.x; t < NC * NC; t += (int)blockDim.x)
            kap_lds[(t / NC) * KS + t % NC] = 1.0 - K[t];
        __syncthreads();
    }
    const int64_t count = stage_count<Item, NC>(c);
    const int lane = (int)__lane_id();
    Grp<NC, G> g;
    g.gi = lane % G;
    g.base = lane - g.gi;
    g.act = g.gi < NC;
    g.row = g.act ? g.gi : NC;
    g.sh = group_dyn + KN + (threadIdx.x / G) * GroupLds<NC, G>::template of<Item>();
    g.vb = g.sh + (Item::kMatrix ? GroupLds<NC, G>::V : 0);
    g.ks = Item::kPerMixture ? nullptr : kap_lds;
    uint32_t(*buf)[kStage] = stage_buf[threadIdx.x / 64];
    int fill[NOUT];
#pragma unroll
    for (int l = 0; l < NOUT; ++l) fill[l] = 0;
    Claim cl(count, (unsigned long long)gridDim.x * (blockDim.x / 64),
             (unsigned long long)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64);
    Item it;
    bool live = false, gone = false;   // the same in every lane of a group
    for (;;) {
        const bool want = !live && !gone;
        const unsigned long long mask = __ballot(want && g.gi == 0);
        if (mask) {
            const unsigned long long rank =
                (unsigned long long)__popcll(mask & lanes_below(g.base));
            const unsigned long long k = cl.next(__popcll(mask), rank, lane, take);
            if (want) {
                if ((int64_t)k < count) live = it.begin(c, stage_id<Item, NC>(c, (int64_t)k), g);
                else gone = true;
            }
        }
        if (__ballot(!gone) == 0ull) break;
        if constexpr (OUT != 0u) it.ob.clear();
        if (live) live = !it.step(c, g);
        if constexpr (OUT != 0u) {
#pragma unroll
            for (int l = 0; l < L_COUNT; ++l) {
                if ((OUT >> l) & 1u) {
                    const int q = slot_of<OUT>(l);
                    stage_slot(c.L, l, it.ob.l0, it.ob.i0, it.ob.n0, buf[q], fill[q], lane);
                    stage_slot(c.L, l, it.ob.l1, it.ob.i1, 1, buf[q], fill[q], lane);
                }
            }
        }
    }
    if constexpr (OUT != 0u) {
#pragma unroll
        for (int l = 0; l < L_COUNT; ++l) {
            if ((OUT >> l) & 1u) {
                const int q = slot_of<OUT>(l);
                if (fill[q] > 0) flush_list(c.L, l, buf[q], fill[q], lane);
            }
        }
    }
}

// Fused form (small batches): a pair of lanes carries one mixture through
// every stage in the staged order, with no lists and no barrier between the
// stages.  The items are those of the staged forms, run back to back; the
// list entries an item's last step produces name the item that runs next.
// The first lane of the pair runs the mixture's items, except that each lane
// runs one of the two stability trials, at the same time.  Every item reads
// and writes only its own mixture's record, so the results are those of the
// staged forms bit for bit; the time is that of the slowest mixture's whole
// path instead of the sum over stages of each stage's slowest item.
template <class Item, int NC>
__device__ __forceinline__ void fused_item(const Ctx<NC> &c, uint32_t id, Outbox &next)
{
    Item it;
    next.clear();
    if (!it.begin(c, id)) return;
    for (;;) {
        it.ob.clear();
        const bool done = it.step(c);
        if (done) {
            next = it.ob;
            return;
        }
    }
}

template <int NC, bool PM>
__global__ void __launch_bounds__(kBlock)
stage_fused(Ctx<NC> c, const double *__restrict__ Tc, const double *__restrict__ Pc,
            const double *__restrict__ om, const double *__restrict__ K)
{
    c.pr = Props{Tc, Pc, om, K};
    // the two lanes of a pair are neighbours in one wavefront
    const int64_t m = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 1;
    const uint32_t t = threadIdx.x & 1u;
    if (m >= c.a.n) return;   // both lanes of the pair
    const uint32_t id = (uint32_t)m;
    Outbox o;
    o.clear();
    if (t == 0) {
        fused_item<FeedItem<NC, PM>, NC>(c, id, o);
        if (o.l0 == L_PRE) fused_item<PreSsItem<NC, PM>, NC>(c, id, o);
    }
    // the first lane's routing, and its record writes, to the second lane
    const int route = __shfl(o.l0, (int)__lane_id() & ~1, 64);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    if (route == L_SA) {
        // trial t in lane t, then the decision (list L_SAFIN) in the first lane
        Outbox q;
        fused_item<SaSsItem<NC, PM>, NC>(c, 2 * id + t, q);
        if (q.l0 == L_SATR) fused_item<SaTrItem<NC, PM>, NC>(c, 2 * id + t, q);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        if (t == 0) fused_item<SaFinItem<NC, PM>, NC>(c, id, o);
    }
    if (t != 0 || c.a.stability_only) return;
    if (o.l0 == L_SPLIT) {
        fused_item<SpSsItem<NC, PM>, NC>(c, id, o);
        if (o.l0 == L_NT || o.l0 == L_NTP) fused_item<SpNtItem<NC, PM>, NC>(c, id, o);
    }
}

// Plain form: begin every item of the stage and list the live ones ...
template <class Item, int NC>
__global__ void __launch_bounds__(kBlock)
stage_plain_begin(Ctx<NC> c, const double *__restrict__ Tc, const double *__restrict__ Pc,
                  const double *__restrict__ om, const double *__restrict__ K, Item *states,
                  uint32_t *active, unsigned long long *nactive)
{
    c.pr = Props{Tc, Pc, om, K};
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= stage_count<Item, NC>(c)) return;
    Item it;
    if (it.begin(c, stage_id<Item, NC>(c, k))) {
        states[k] = it;
        active[atomicAdd(nactive, 1ull)] = (uint32_t)k;
    }
}

// ... then one step of every live item per launch, listing those still live
// (the list order does not matter: each item's result depends on its own
// state only).
template <class Item, int NC>
__global__ void __launch_bounds__(kBlock)
stage_plain_step(Ctx<NC> c, const double *__restrict__ Tc, const double *__restrict__ Pc,
                 const double *__restrict__ om, const double *__restrict__ K, Item *states,
                 const uint32_t *__restrict__ active, int64_t nact, uint32_t *next,
                 unsigned long long *nnext)
{
    c.pr = Props{Tc, Pc, om, K};
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nact) return;
    const uint32_t k = active[j];
    Item it = states[k];
    it.ob.clear();
    const bool done = it.step(c);
    const int lane = (int)__lane_id();
#pragma unroll
    for (int l = 0; l < L_COUNT; ++l) {
        append_slot(c.L, l, it.ob.l0, it.ob.i0, it.ob.n0, lane);
        append_slot(c.L, l, it.ob.l1, it.ob.i1, 1, lane);
    }
    if (!done) {
        states[k] = it;
        next[atomicAdd(nnext, 1ull)] = k;
    }
}

// Diagnostic: ln phi, Z and the full Phi matrix at given compositions.
template <int NC>
__global__ void __launch_bounds__(kBlock)
eval_phase_kernel(int64_t n, const double *__restrict__ c, const double *__restrict__ T,
                  const double *__restrict__ P, const double *__restrict__ Tc,
                  const double *__restrict__ Pc, const double *__restrict__ om,
                  const double *__restrict__ K, double *lnphi, double *Zo, double *phi)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    Eos<NC> e;
    eos_setup<NC>(e, Tc, Pc, om, T[m], P[m]);
    double w[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) w[i] = c[m * NC + i];
    Phase<NC> o;
    uint32_t fl = 0;
    phase_eval<NC>(o, e, K, w, fl);
#pragma unroll
    for (int i = 0; i < NC; ++i) lnphi[m * NC + i] = o.lnphi[i];
    Zo[m] = o.Z;
    if (phi) {
        double F[Tri<NC>::N];
        phase_derivs<NC>(F, o, e, K, fl);
#pragma unroll
        for (int i = 0; i < NC; ++i)
#pragma unroll
            for (int j = 0; j <= i; ++j) {
                phi[m * NC * NC + i * NC + j] = F[tri(i, j)];
                phi[m * NC * NC + j * NC + i] = F[tri(i, j)];
            }
    }
}

// ---------------------------------------------------------------------------
// Backward (implicit function theorem on the converged split)
// ---------------------------------------------------------------------------


template <int NC, bool PM>
__global__ void __launch_bounds__(kBlock)
flash_backward_kernel(BwdArgs a, const double *__restrict__ Tc0, const double *__restrict__ Pc0,
                      const double *__restrict__ om0, const double *__restrict__ K0)
{
    constexpr int NP = Tri<NC>::N;
    constexpr int NQ = NC * (NC - 1) / 2;
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= a.n) return;
    const Props pp = mix_props<NC, PM>(Props{Tc0, Pc0, om0, K0}, m);
    const double *__restrict__ Tc = pp.Tc;
    const double *__restrict__ Pc = pp.Pc;
    const double *__restrict__ om = pp.om;
    const double *__restrict__ K = pp.K;
    double zt[NC], s = 0.0;
#pragma unroll
    for (int i = 0; i < NC; ++i) { zt[i] = a.z[m * NC + i]; s += zt[i]; }
#pragma unroll
    for (int i = 0; i < NC; ++i) zt[i] /= s;
    const uint16_t st = a.status ? a.status[m] : (uint16_t)0;
    double ztb[NC], gT = 0.0, gP = 0.0;
    double gkq[NQ > 0 ? NQ : 1];
#pragma unroll
    for (int q = 0; q < NQ; ++q) gkq[q] = 0.0;
    bool bad = (st & (kStInvalid | kStSplitUnconv | kStStepCap)) != 0;
    if (!bad && a.label[m] == 1) {
        const double T = a.T[m], P = a.P[m], beta = a.beta[m];
        double x[NC], y[NC], gx[NC], gy[NC];
        double gxx = 0.0, gyy = 0.0;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            x[i] = a.x[m * NC + i];
            y[i] = a.y[m * NC + i];
            gx[i] = a.gx[m * NC + i];
            gy[i] = a.gy[m * NC + i];
            gxx += gx[i] * x[i];
            gyy += gy[i] * y[i];
        }
        const double gb = a.gb[m];
        // u_bar = (do/du)^T o_bar for o = (beta = sum u, y = u/beta,
        // x = (z~ - u)/(1 - beta))
        double lam[NC];
        const double ib = 1.0 / beta, il = 1.0 / (1.0 - beta);
#pragma unroll
        for (int j = 0; j < NC; ++j) lam[j] = gb + (gy[j] - gyy) * ib - (gx[j] - gxx) * il;
        // H~ lambda = u_bar with the forward's factor H~ = L L^T
        double Lf[NP], dinv[NC], tmp[NC];
#pragma unroll
        for (int k = 0; k < NP; ++k) Lf[k] = a.factor[m * NP + k];
#pragma unroll
        for (int i = 0; i < NC; ++i) dinv[i] = 1.0 / Lf[tri(i, i)];
        lower_solve<NC>(tmp, Lf, dinv, lam);
        upper_solve<NC>(lam, Lf, dinv, tmp);
        bad = !isfinite(lam[0]);
        // phase data at the solution
        Eos<NC> e;
        eos_setup<NC>(e, Tc, Pc, om, T, P);
        uint32_t fl = 0;
        Phase<NC> oL, oV;
        phase_eval<NC>(oL, e, K, x, fl);
        double Phi[NP];
        phase_derivs<NC>(Phi, oL, e, K, fl);
        // z~_bar_j = [gx_j + lambda_j/x_j - sum lambda + (Phi^L lambda)_j]/(1 - beta)
        double sl = 0.0;
#pragma unroll
        for (int i = 0; i < NC; ++i) sl += lam[i];
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            double pl = 0.0;
#pragma unroll
            for (int i = 0; i < NC; ++i) pl += Phi[i >= j ? tri(i, j) : tri(j, i)] * lam[i];
            ztb[j] = (gx[j] + lam[j] / x[j] - sl + pl) * il;
        }
        PhaseGrad<NC> gL, gV;
        phase_param_vjp<NC>(gL, oL, e, x, lam, K, Tc, om, T, P);
        phase_eval<NC>(oV, e, K, y, fl);
        phase_param_vjp<NC>(gV, oV, e, y, lam, K, Tc, om, T, P);
        gT = -(gV.dT - gL.dT);
        gP = -(gV.dP - gL.dP);
#pragma unroll
        for (int q = 0; q < NQ; ++q) gkq[q] = -(gV.dk[q] - gL.dk[q]);
    } else if (!bad) {
        // single phase: x = y = z~
#pragma unroll
        for (int i = 0; i < NC; ++i) ztb[i] = a.gx[m * NC + i] + a.gy[m * NC + i];
    }
    if (bad) {
        const double nan = __builtin_nan("");
#pragma unroll
        for (int i = 0; i < NC; ++i) ztb[i] = nan;
        gT = gP = nan;
#pragma unroll
        for (int q = 0; q < NQ; ++q) gkq[q] = nan;
    }
    // through the normalisation z~ = z / sum z
    double zz = 0.0;
#pragma unroll
    for (int i = 0; i < NC; ++i) zz += ztb[i] * zt[i];
#pragma unroll
    for (int j = 0; j < NC; ++j) a.gz[m * NC + j] = (ztb[j] - zz) / s;
    a.gT[m] = gT;
    a.gP[m] = gP;
    if (a.gk) {
        int q = 0;
#pragma unroll
        for (int i = 0; i < NC; ++i) a.gk[m * NC * NC + i * NC + i] = bad ? gT /* NaN */ : 0.0;
#pragma unroll
        for (int i = 0; i < NC; ++i)
#pragma unroll
            for (int j = i + 1; j < NC; ++j, ++q) {
                a.gk[m * NC * NC + i * NC + j] = 0.5 * gkq[q];
                a.gk[m * NC * NC + j * NC + i] = 0.5 * gkq[q];
            }
    }
    if (a.kpart) {
        // unconverged mixtures (NaN above) do not enter the batch sum
#pragma unroll
        for (int q = 0; q < NQ; ++q) a.kpart[(int64_t)q * a.n + m] = bad ? 0.0 : gkq[q];
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

// Resident blocks of one kernel on the current device (blocks per CU times
// CUs) for a block size and dynamic LDS bytes, queried once per kernel,
// device and block size and then kept.
int resident_blocks(const void *kernel, int block, size_t lds = 0)
{
    struct Entry {
        const void *kernel;
        int dev, block, blocks;
    };
    static std::mutex mu;
    static std::vector<Entry> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    {
        std::lock_guard<std::mutex> lk(mu);
        for (const Entry &e : cache)
            if (e.kernel == kernel && e.dev == dev && e.block == block) return e.blocks;
    }
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        return -1;
    const int blocks = (per_cu > 0 ? per_cu : 1) * cus;
    std::lock_guard<std::mutex> lk(mu);
    cache.push_back(Entry{kernel, dev, block, blocks});
    return blocks;
}


// Workspace: counters | per-mixture records | stage lists | (plain form:)
// item states and two active lists.
constexpr int kNumStages = 7;
constexpr int kNumCounters = 16;   // L_COUNT list counts, kNumStages take counters, 2 plain
constexpr int kTake0 = L_COUNT;
constexpr int kPlain0 = L_COUNT + kNumStages;
static_assert(kPlain0 + 2 <= kNumCounters, "counter block too small");
constexpr size_t kCounterBytes = (size_t)kNumCounters * kCounterStride * 8;

template <int NC>
size_t plain_state_bytes()
{
    size_t m = sizeof(FeedItem<NC, false>);
    m = m > sizeof(PreSsItem<NC, false>) ? m : sizeof(PreSsItem<NC, false>);
    m = m > sizeof(SaSsItem<NC, false>) ? m : sizeof(SaSsItem<NC, false>);
    m = m > sizeof(SaTrItem<NC, false>) ? m : sizeof(SaTrItem<NC, false>);
    m = m > sizeof(SaFinItem<NC, false>) ? m : sizeof(SaFinItem<NC, false>);
    m = m > sizeof(SpSsItem<NC, false>) ? m : sizeof(SpSsItem<NC, false>);
    m = m > sizeof(SpNtItem<NC, false>) ? m : sizeof(SpNtItem<NC, false>);
    return m;
}

template <int NC>
size_t workspace_bytes(int64_t n, int form)
{
    const size_t un = (size_t)n;
    size_t b = kCounterBytes + align256(un * sizeof(MixRec<NC>)) + 3 * align256(2 * un * 4) +
               4 * align256(un * 4);
    if (form == PTFLASH_FORM_PLAIN)
        b += align256(2 * un * plain_state_bytes<NC>()) + 2 * align256(2 * un * 4);
    return b;
}

struct Carve {
    char *p;
    template <typename T>
    T *take(size_t bytes)
    {
        T *r = (T *)p;
        p += align256(bytes);
        return r;
    }
};

template <int NC>
void setup_ctx(Ctx<NC> &c, const FlashArgs &a, int64_t n, void *ws, char **tail)
{
    Carve cv{(char *)ws};
    c.a = a;
    c.pr = Props{nullptr, nullptr, nullptr, nullptr};
    unsigned long long *cnt = cv.take<unsigned long long>(kCounterBytes);
    c.rec = cv.take<MixRec<NC>>((size_t)n * sizeof(MixRec<NC>));
    c.L.ids[L_SA] = cv.take<uint32_t>(2 * (size_t)n * 4);
    c.L.ids[L_SATR] = cv.take<uint32_t>(2 * (size_t)n * 4);
    c.L.ids[L_PRE] = cv.take<uint32_t>(2 * (size_t)n * 4);
    c.L.ids[L_SAFIN] = cv.take<uint32_t>((size_t)n * 4);
    c.L.ids[L_SPLIT] = cv.take<uint32_t>((size_t)n * 4);
    c.L.ids[L_NT] = cv.take<uint32_t>((size_t)n * 4);
    c.L.ids[L_NTP] = cv.take<uint32_t>((size_t)n * 4);
    c.L.count = cnt;
    *tail = cv.p;
}

// Grid of a persistent stage: the requested size, else every block the
// device holds at once, but no more blocks than it takes to give each of
// the stage's items (at most two per mixture: the two stability trials)
// its lanes, so that a small batch runs on few wavefronts.
int grid_for(const void *kernel, int block, int requested, int64_t n, int lanes_per_item,
             size_t lds = 0)
{
    if (requested > 0) return requested;
    const int full = resident_blocks(kernel, block, lds);
    if (full <= 0) return -1;
    const int64_t need = (2 * n * lanes_per_item + block - 1) / block;
    return (int)(need < 1 ? 1 : need < full ? need : full);
}

template <class Item, int NC>
int run_persistent_stage(const Ctx<NC> &c, const ptflash_problem *p,
                                const ptflash_options *o, int take_slot, hipStream_t s)
{
    const int block = o->block > 0 ? o->block : tuned_block(NC, Item::kPerMixture);
    if (block % 64 != 0 || block > kBlock) return PTFLASH_EINVAL;
    const int grid = grid_for((const void *)stage_persistent<Item, NC>, block, o->grid, p->n, 1);
    if (grid <= 0) return PTFLASH_EHIP;
    hipLaunchKernelGGL((stage_persistent<Item, NC>), dim3(grid), dim3(block), 0, s, c, p->Tc,
                       p->Pc, p->omega, p->kij, c.L.cnt(take_slot));
    return hipGetLastError() == hipSuccess ? PTFLASH_OK : PTFLASH_EHIP;
}

// Dynamic LDS bytes of a group stage block of the given size.
template <class Item, int NC, int G>
size_t group_lds_bytes(int block)
{
    const size_t kn = Item::kPerMixture ? 0 : (size_t)NC * KapLds::stride<NC>();
    return 8 * (kn + (size_t)(block / G) * GroupLds<NC, G>::template of<Item>());
}

template <class Item, int NC, int G>
int run_persistent_stage_group(const Ctx<NC> &c, const ptflash_problem *p,
                               const ptflash_options *o, int take_slot, hipStream_t s)
{
    const int block = o->block > 0 ? o->block : tuned_block(NC, Item::kPerMixture);
    if (block % 64 != 0 || block > kBlock) return PTFLASH_EINVAL;
    const size_t lds = group_lds_bytes<Item, NC, G>(block);
    int dev = 0, lds_max = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
            hipSuccess)
        return PTFLASH_EHIP;
    if (lds > (size_t)lds_max) return PTFLASH_EINVAL;   // a smaller block fits
    const int grid = grid_for((const void *)stage_persistent_group<Item, NC, G>, block, o->grid,
                              p->n, G, lds);
    if (grid <= 0) return PTFLASH_EHIP;
    hipLaunchKernelGGL((stage_persistent_group<Item, NC, G>), dim3(grid), dim3(block), lds, s, c,
                       p->Tc, p->Pc, p->omega, p->kij, c.L.cnt(take_slot));
    return hipGetLastError() == hipSuccess ? PTFLASH_OK : PTFLASH_EHIP;
}

// Lanes per mixture of a trust-region stage, or 0 when l is not available
// for this nc.
template <int NC>
int lanes_ok(int l)
{
    if (l == 1) return 1;
    if (NC < kGroupMinNc) return 0;
    if (l == 16 && NC <= 16) return 16;
    if (l == 32 && NC <= 32) return 32;
    return 0;
}

// The stability trust region: the option, or the tuned choice for this nc
// and layout of the component sets (pm: one set per mixture).
template <int NC>
int lanes_sa(const ptflash_options *o, bool pm)
{
    return lanes_ok<NC>(o->lanes_per_mixture > 0 ? o->lanes_per_mixture
                                                 : tuned_lanes_sa(NC, pm));
}

// The split trust region: lanes_split, else lanes_per_mixture, else tuned.
template <int NC>
int lanes_sp(const ptflash_options *o, bool pm)
{
    const int l = o->lanes_split > 0 ? o->lanes_split
                  : o->lanes_per_mixture > 0 ? o->lanes_per_mixture : tuned_lanes_sp(NC, pm);
    return lanes_ok<NC>(l);
}

// The two substitution stages: lanes_ss, else tuned.
template <int NC>
int lanes_ss(const ptflash_options *o, bool pm)
{
    return lanes_ok<NC>(o->lanes_ss > 0 ? o->lanes_ss : tuned_lanes_ss(NC, pm));
}

// One stage with a group form (Item1: one mixture per lane; ItemG<G>:
// groups).
template <template <int, bool> class Item1, template <int, bool, int> class ItemG, int NC,
          bool PM>
int run_tr_stage(const Ctx<NC> &c, const ptflash_problem *p, const ptflash_options *o,
                 int lanes, int take_slot, hipStream_t s)
{
    if constexpr (NC >= kGroupMinNc && NC <= 16) {
        if (lanes == 16)
            return run_persistent_stage_group<ItemG<NC, PM, 16>, NC, 16>(c, p, o, take_slot, s);
    }
    if constexpr (NC >= kGroupMinNc && NC <= 32) {
        if (lanes == 32)
            return run_persistent_stage_group<ItemG<NC, PM, 32>, NC, 32>(c, p, o, take_slot, s);
    }
    if (lanes == 1) return run_persistent_stage<Item1<NC, PM>, NC>(c, p, o, take_slot, s);
    return PTFLASH_EINVAL;
}

template <int NC, bool PM>
int launch_persistent(const FlashArgs &a, const ptflash_problem *p, const ptflash_options *o,
                      void *ws, hipStream_t s)
{
    const int lsa = lanes_sa<NC>(o, PM), lsp = lanes_sp<NC>(o, PM), lss = lanes_ss<NC>(o, PM);
    if (lsa == 0 || lsp == 0 || lss == 0) return PTFLASH_EINVAL;
    Ctx<NC> c;
    char *tail;
    setup_ctx<NC>(c, a, p->n, ws, &tail);
    hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, s, c.L.count, kNumCounters);
    int rc;
    if ((rc = run_persistent_stage<FeedItem<NC, PM>, NC>(c, p, o, kTake0 + 0, s))) return rc;
    if ((rc = run_persistent_stage<PreSsItem<NC, PM>, NC>(c, p, o, kTake0 + 1, s))) return rc;
    if ((rc = run_tr_stage<SaSsItem, SaSsGroup, NC, PM>(c, p, o, lss, kTake0 + 2, s))) return rc;
    if ((rc = run_tr_stage<SaTrItem, SaTrGroup, NC, PM>(c, p, o, lsa, kTake0 + 3, s))) return rc;
    if ((rc = run_persistent_stage<SaFinItem<NC, PM>, NC>(c, p, o, kTake0 + 4, s))) return rc;
    if (a.stability_only) return PTFLASH_OK;
    if ((rc = run_tr_stage<SpSsItem, SpSsGroup, NC, PM>(c, p, o, lss, kTake0 + 5, s))) return rc;
    if ((rc = run_tr_stage<SpNtItem, SpNtGroup, NC, PM>(c, p, o, lsp, kTake0 + 6, s))) return rc;
    return PTFLASH_OK;
}

// Reads a device counter after the work queued so far (host sync).
int read_count(const unsigned long long *dcnt, int64_t &out, hipStream_t s)
{
    unsigned long long h = 0;
    if (hipGetLastError() != hipSuccess) return PTFLASH_EHIP;
    if (hipMemcpyAsync(&h, dcnt, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return PTFLASH_EHIP;
    out = (int64_t)h;
    return PTFLASH_OK;
}

template <class Item, int NC>
int run_plain_stage(const Ctx<NC> &c, const ptflash_problem *p, char *tail, hipStream_t s)
{
    const int64_t n = p->n;
    Carve cv{tail};
    Item *states = cv.take<Item>(2 * (size_t)n * plain_state_bytes<NC>());
    uint32_t *la = cv.take<uint32_t>(2 * (size_t)n * 4);
    uint32_t *lb = cv.take<uint32_t>(2 * (size_t)n * 4);
    unsigned long long *na = c.L.cnt(kPlain0), *nb = c.L.cnt(kPlain0 + 1);
    int64_t count = n;
    int rc;
    if (Item::LIST >= 0 && (rc = read_count(c.L.cnt(Item::LIST), count, s))) return rc;
    if (Item::LIST2 >= 0) {
        int64_t c2 = 0;
        if ((rc = read_count(c.L.cnt(Item::LIST2 < 0 ? 0 : Item::LIST2), c2, s))) return rc;
        count += c2;
    }
    if (count == 0) return PTFLASH_OK;
    auto grid = [](int64_t k) { return dim3((unsigned)((k + kBlock - 1) / kBlock)); };
    hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, s, na, 1);
    hipLaunchKernelGGL((stage_plain_begin<Item, NC>), grid(count), dim3(kBlock), 0, s, c, p->Tc,
                       p->Pc, p->omega, p->kij, states, la, na);
    int64_t nact = 0;
    if ((rc = read_count(na, nact, s))) return rc;
    for (int guard = 0; nact > 0 && guard <= kStepGuard + 1; ++guard) {
        hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, s, nb, 1);
        hipLaunchKernelGGL((stage_plain_step<Item, NC>), grid(nact), dim3(kBlock), 0, s, c, p->Tc,
                           p->Pc, p->omega, p->kij, states, la, nact, lb, nb);
        if ((rc = read_count(nb, nact, s))) return rc;
        uint32_t *t = la; la = lb; lb = t;
        unsigned long long *tc = na; na = nb; nb = tc;
    }
    return PTFLASH_OK;
}

template <int NC, bool PM>
int launch_fused(const FlashArgs &a, const ptflash_problem *p, const ptflash_options *o,
                 void *ws, hipStream_t s)
{
    const int block = o->block > 0 ? o->block : 64;
    if (block % 64 != 0 || block > kBlock) return PTFLASH_EINVAL;
    Ctx<NC> c;
    char *tail;
    setup_ctx<NC>(c, a, p->n, ws, &tail);
    const int64_t blocks = (2 * p->n + block - 1) / block;   // two lanes per mixture
    if (blocks > 0)
        hipLaunchKernelGGL((stage_fused<NC, PM>), dim3((unsigned)blocks), dim3(block), 0, s, c,
                           p->Tc, p->Pc, p->omega, p->kij);
    return hipGetLastError() == hipSuccess ? PTFLASH_OK : PTFLASH_EHIP;
}

template <int NC, bool PM>
int launch_plain(const FlashArgs &a, const ptflash_problem *p, void *ws, hipStream_t s)
{
    Ctx<NC> c;
    char *tail;
    setup_ctx<NC>(c, a, p->n, ws, &tail);
    hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, s, c.L.count, kNumCounters);
    int rc;
    if ((rc = run_plain_stage<FeedItem<NC, PM>, NC>(c, p, tail, s))) return rc;
    if ((rc = run_plain_stage<PreSsItem<NC, PM>, NC>(c, p, tail, s))) return rc;
    if ((rc = run_plain_stage<SaSsItem<NC, PM>, NC>(c, p, tail, s))) return rc;
    if ((rc = run_plain_stage<SaTrItem<NC, PM>, NC>(c, p, tail, s))) return rc;
    if ((rc = run_plain_stage<SaFinItem<NC, PM>, NC>(c, p, tail, s))) return rc;
    if (a.stability_only) return PTFLASH_OK;
    if ((rc = run_plain_stage<SpSsItem<NC, PM>, NC>(c, p, tail, s))) return rc;
    if ((rc = run_plain_stage<SpNtItem<NC, PM>, NC>(c, p, tail, s))) return rc;
    return PTFLASH_OK;
}

template <int NC>
int launch_eval(int64_t n, const double *c, const double *T, const double *P,
                       const double *Tc, const double *Pc, const double *om, const double *K,
                       double *lnphi, double *Z, double *phi, hipStream_t s)
{
    const int64_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 0)
        hipLaunchKernelGGL(eval_phase_kernel<NC>, dim3((unsigned)blocks), dim3(kBlock), 0, s, n,
                           c, T, P, Tc, Pc, om, K, lnphi, Z, phi);
    return hipGetLastError() == hipSuccess ? PTFLASH_OK : PTFLASH_EHIP;
}

}  // namespace

template <int NC>
size_t nc_workspace_bytes(int64_t n, int form)
{
    return workspace_bytes<NC>(n, form);
}

// Batches up to this many mixtures run the persistent form as one fused
// launch unless the caller sets its launch shape (grid, block or lanes per
// mixture): below it the staged form's time is the sum of its stages'
// slowest items, which the fused form's slowest whole path undercuts.  The
// fused form keeps a whole mixture on one lane pair, so from nc ~ 12, where
// the staged form moves the trust-region work onto lane groups, it pays off
// only for smaller batches (gfx950, measured at nc 3, 5, 8, 12, 16 and 20).
template <int NC>
constexpr int64_t fused_max_n()
{
    return NC <= 8 ? 150000 : 400000 / NC;
}

template <int NC, bool PM>
int nc_flash_pm(const FlashArgs &a, const ptflash_problem *p, const ptflash_options *o, void *ws,
                hipStream_t s)
{
    if (o->form == PTFLASH_FORM_PLAIN) return launch_plain<NC, PM>(a, p, ws, s);
    if (o->form == PTFLASH_FORM_FUSED) return launch_fused<NC, PM>(a, p, o, ws, s);
    if (o->grid <= 0 && o->block <= 0 && o->lanes_per_mixture <= 0 && o->lanes_split <= 0 &&
        o->lanes_ss <= 0 && p->n <= fused_max_n<NC>()) {
        ptflash_options f = *o;
        f.block = 64;
        return launch_fused<NC, PM>(a, p, &f, ws, s);
    }
    return launch_persistent<NC, PM>(a, p, o, ws, s);
}

template <int NC, bool PM>
int nc_backward_pm(const BwdArgs &b, const ptflash_problem *p, hipStream_t s)
{
    const unsigned nb = (unsigned)((p->n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((flash_backward_kernel<NC, PM>), dim3(nb), dim3(kBlock), 0, s, b, p->Tc,
                       p->Pc, p->omega, p->kij);
    return hipGetLastError() == hipSuccess ? PTFLASH_OK : PTFLASH_EHIP;
}

template <int NC>
int nc_eval(int64_t n, const double *c, const double *T, const double *P, const double *Tc,
            const double *Pc, const double *om, const double *K, double *lnphi, double *Z,
            double *phi, hipStream_t s)
{
    return launch_eval<NC>(n, c, T, P, Tc, Pc, om, K, lnphi, Z, phi, s);
}

}  // namespace ptf
