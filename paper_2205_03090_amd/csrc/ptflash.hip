// ptflash.hip -- kernels and C ABI of the gfx950 SRK PT flash.
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
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "ptflash.h"
#include "flash_stages.hpp"
#include "adjoint_device.hpp"

namespace ptf {

constexpr int kMinNc = 2;
constexpr int kMaxNc = PTF_MAX_NC;
constexpr int kBlock = 256;

__global__ void reset_counters(unsigned long long *q, int n)
{
    if ((int)threadIdx.x < n) q[threadIdx.x] = 0ull;
}

// Number of items of a stage: all mixtures for the first stage, else the
// length of the stage's list (written by the previous stages).
template <class Item, int NC>
__device__ __forceinline__ int64_t stage_count(const Ctx<NC> &c)
{
    return Item::LIST < 0 ? c.a.n : (int64_t)c.L.count[Item::LIST];
}

template <class Item, int NC>
__device__ __forceinline__ uint32_t stage_id(const Ctx<NC> &c, int64_t k)
{
    return Item::LIST < 0 ? (uint32_t)k : c.L.ids[Item::LIST < 0 ? 0 : Item::LIST][k];
}

// Persistent stage: one item per lane; lanes whose item finished take the
// next indices from *take (one atomic per wavefront and step).  Every item
// finishes within its stage's iteration caps (and kStepGuard steps), so every
// wavefront reaches the exit.
template <class Item, int NC>
__global__ void __launch_bounds__(kBlock)
stage_persistent(Ctx<NC> c, const double *__restrict__ Tc, const double *__restrict__ Pc,
                 const double *__restrict__ om, const double *__restrict__ K,
                 unsigned long long *__restrict__ take)
{
    c.pr = Props{Tc, Pc, om, K};
    const int64_t count = stage_count<Item, NC>(c);
    Item it;
    bool live = false, gone = false;
    const int lane = (int)__lane_id();
    for (;;) {
        const bool want = !live && !gone;
        const unsigned long long mask = __ballot(want);
        if (mask) {
            const int leader = __ffsll((unsigned long long)mask) - 1;
            unsigned long long base = 0;
            if (lane == leader) base = atomicAdd(take, (unsigned long long)__popcll(mask));
            const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)base, leader);
            const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(base >> 32), leader);
            base = ((unsigned long long)hi << 32) | lo;
            if (want) {
                const unsigned long long below = mask & ((1ull << lane) - 1ull);
                const int64_t k = (int64_t)(base + (unsigned long long)__popcll(below));
                if (k < count) live = it.begin(c, stage_id<Item, NC>(c, k));
                else gone = true;
            }
        }
        if (__ballot(!gone) == 0ull) break;
        if (live) live = !it.step(c);
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
    if (!it.step(c)) {
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

struct BwdArgs {
    int64_t n;
    const double *z, *T, *P;
    const int8_t *label;
    const double *beta, *x, *y, *factor;
    const uint16_t *status;
    const double *gb, *gx, *gy;
    double *gz, *gT, *gP;
    double *gk;        // n*nc*nc (per mixture) or NULL when reduced
    double *kpart;     // npair*n contributions (pair-major) when reduced
};

template <int NC>
__global__ void __launch_bounds__(kBlock)
flash_backward_kernel(BwdArgs a, const double *__restrict__ Tc, const double *__restrict__ Pc,
                      const double *__restrict__ om, const double *__restrict__ K)
{
    constexpr int NP = Tri<NC>::N;
    constexpr int NQ = NC * (NC - 1) / 2;
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= a.n) return;
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

// Deterministic batch sum of the k contributions: one block per pair, each
// thread sums a fixed strided subset in order, then a fixed tree in LDS.
__global__ void __launch_bounds__(kBlock)
reduce_pairs(const double *__restrict__ kpart, int64_t n, int nc, double *gk)
{
    __shared__ double red[kBlock];
    const int q = blockIdx.x;
    double acc = 0.0;
    for (int64_t m = threadIdx.x; m < n; m += kBlock) acc += kpart[(int64_t)q * n + m];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        // pair index -> (i, j), i < j
        int i = 0, r = q;
        while (r >= nc - 1 - i) { r -= nc - 1 - i; ++i; }
        const int j = i + 1 + r;
        gk[i * nc + j] = 0.5 * red[0];
        gk[j * nc + i] = 0.5 * red[0];
        if (q == 0)
            for (int d = 0; d < nc; ++d) gk[d * nc + d] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

static int device_cus()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return cus;
}

static void fill_args(FlashArgs &a, const ptflash_problem *p, const ptflash_options *o,
                      const ptflash_result *r)
{
    a.n = p->n;
    a.z = p->z;
    a.T = p->T;
    a.P = p->P;
    a.max_pre_ss = o->max_pre_ss;
    a.max_ss = o->max_ss;
    a.max_tr_sa = o->max_tr_sa;
    a.max_tr_split = o->max_tr_split;
    a.max_polish = o->max_polish;
    a.dem_every = o->dem_every;
    a.keep_factor = o->keep_factor;
    a.tol_sa_ss = o->tol_sa_ss;
    a.tol_sa_tr = o->tol_sa_tr;
    a.tol_split_ss = o->tol_split_ss;
    a.tol_split_tr = o->tol_split_tr;
    a.tol_polish = o->tol_polish;
    a.eps_tm = o->eps_tm;
    a.label = r->label;
    a.beta = r->beta;
    a.x = r->x;
    a.y = r->y;
    a.iters = r->iters;
    a.status = r->status;
    a.flops = r->flops;
    a.factor = r->factor;
}

static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace: counters | per-mixture records | stage lists | (plain form:)
// item states and two active lists.
constexpr int kNumCounters = 16;   // L_COUNT list counts, 6 take counters, 2 plain
constexpr int kTake0 = L_COUNT;
constexpr int kPlain0 = L_COUNT + 6;

template <int NC>
static size_t plain_state_bytes()
{
    size_t m = sizeof(PreItem<NC>);
    m = m > sizeof(SaSsItem<NC>) ? m : sizeof(SaSsItem<NC>);
    m = m > sizeof(SaTrItem<NC>) ? m : sizeof(SaTrItem<NC>);
    m = m > sizeof(SaFinItem<NC>) ? m : sizeof(SaFinItem<NC>);
    m = m > sizeof(SpSsItem<NC>) ? m : sizeof(SpSsItem<NC>);
    m = m > sizeof(SpNtItem<NC>) ? m : sizeof(SpNtItem<NC>);
    return m;
}

template <int NC>
static size_t workspace_bytes(int64_t n, int form)
{
    const size_t un = (size_t)n;
    size_t b = 256 + align256(un * sizeof(MixRec<NC>)) + 3 * align256(2 * un * 4) +
               3 * align256(un * 4);
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
static void setup_ctx(Ctx<NC> &c, const FlashArgs &a, int64_t n, void *ws, char **tail)
{
    Carve cv{(char *)ws};
    c.a = a;
    c.pr = Props{nullptr, nullptr, nullptr, nullptr};
    unsigned long long *cnt = cv.take<unsigned long long>(256);
    c.rec = cv.take<MixRec<NC>>((size_t)n * sizeof(MixRec<NC>));
    c.L.ids[L_SA] = cv.take<uint32_t>(2 * (size_t)n * 4);
    c.L.ids[L_SATR] = cv.take<uint32_t>(2 * (size_t)n * 4);
    cv.take<uint32_t>(2 * (size_t)n * 4);   // spare (keeps the layout aligned to the size formula)
    c.L.ids[L_SAFIN] = cv.take<uint32_t>((size_t)n * 4);
    c.L.ids[L_SPLIT] = cv.take<uint32_t>((size_t)n * 4);
    c.L.ids[L_NT] = cv.take<uint32_t>((size_t)n * 4);
    c.L.count = cnt;
    *tail = cv.p;
}

static int grid_for(const void *kernel, int block, int requested)
{
    if (requested > 0) return requested;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess)
        return -1;
    const int cus = device_cus();
    if (cus <= 0) return -1;
    return (per_cu > 0 ? per_cu : 1) * cus;
}

template <class Item, int NC>
static int run_persistent_stage(const Ctx<NC> &c, const ptflash_problem *p,
                                const ptflash_options *o, int take_slot, hipStream_t s)
{
    const int block = o->block > 0 ? o->block : kBlock;
    if (block % 64 != 0 || block > kBlock) return PTFLASH_EINVAL;
    const int grid = grid_for((const void *)stage_persistent<Item, NC>, block, o->grid);
    if (grid <= 0) return PTFLASH_EHIP;
    hipLaunchKernelGGL((stage_persistent<Item, NC>), dim3(grid), dim3(block), 0, s, c, p->Tc,
                       p->Pc, p->omega, p->kij, c.L.count + take_slot);
    return hipGetLastError() == hipSuccess ? PTFLASH_OK : PTFLASH_EHIP;
}

template <int NC>
static int launch_persistent(const FlashArgs &a, const ptflash_problem *p,
                             const ptflash_options *o, void *ws, hipStream_t s)
{
    Ctx<NC> c;
    char *tail;
    setup_ctx<NC>(c, a, p->n, ws, &tail);
    hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, s, c.L.count, kNumCounters);
    int rc;
    if ((rc = run_persistent_stage<PreItem<NC>, NC>(c, p, o, kTake0 + 0, s))) return rc;
    if ((rc = run_persistent_stage<SaSsItem<NC>, NC>(c, p, o, kTake0 + 1, s))) return rc;
    if ((rc = run_persistent_stage<SaTrItem<NC>, NC>(c, p, o, kTake0 + 2, s))) return rc;
    if ((rc = run_persistent_stage<SaFinItem<NC>, NC>(c, p, o, kTake0 + 3, s))) return rc;
    if ((rc = run_persistent_stage<SpSsItem<NC>, NC>(c, p, o, kTake0 + 4, s))) return rc;
    if ((rc = run_persistent_stage<SpNtItem<NC>, NC>(c, p, o, kTake0 + 5, s))) return rc;
    return PTFLASH_OK;
}

// Reads a device counter after the work queued so far (host sync).
static int read_count(const unsigned long long *dcnt, int64_t &out, hipStream_t s)
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
static int run_plain_stage(const Ctx<NC> &c, const ptflash_problem *p, char *tail, hipStream_t s)
{
    const int64_t n = p->n;
    Carve cv{tail};
    Item *states = cv.take<Item>(2 * (size_t)n * plain_state_bytes<NC>());
    uint32_t *la = cv.take<uint32_t>(2 * (size_t)n * 4);
    uint32_t *lb = cv.take<uint32_t>(2 * (size_t)n * 4);
    unsigned long long *na = c.L.count + kPlain0, *nb = c.L.count + kPlain0 + 1;
    int64_t count = n;
    int rc;
    if (Item::LIST >= 0 && (rc = read_count(c.L.count + Item::LIST, count, s))) return rc;
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

template <int NC>
static int launch_plain(const FlashArgs &a, const ptflash_problem *p, void *ws, hipStream_t s)
{
    Ctx<NC> c;
    char *tail;
    setup_ctx<NC>(c, a, p->n, ws, &tail);
    hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, s, c.L.count, kNumCounters);
    int rc;
    if ((rc = run_plain_stage<PreItem<NC>, NC>(c, p, tail, s))) return rc;
    if ((rc = run_plain_stage<SaSsItem<NC>, NC>(c, p, tail, s))) return rc;
    if ((rc = run_plain_stage<SaTrItem<NC>, NC>(c, p, tail, s))) return rc;
    if ((rc = run_plain_stage<SaFinItem<NC>, NC>(c, p, tail, s))) return rc;
    if ((rc = run_plain_stage<SpSsItem<NC>, NC>(c, p, tail, s))) return rc;
    if ((rc = run_plain_stage<SpNtItem<NC>, NC>(c, p, tail, s))) return rc;
    return PTFLASH_OK;
}

template <int NC>
static int launch_eval(int64_t n, const double *c, const double *T, const double *P,
                       const double *Tc, const double *Pc, const double *om, const double *K,
                       double *lnphi, double *Z, double *phi, hipStream_t s)
{
    const int64_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 0)
        hipLaunchKernelGGL(eval_phase_kernel<NC>, dim3((unsigned)blocks), dim3(kBlock), 0, s, n,
                           c, T, P, Tc, Pc, om, K, lnphi, Z, phi);
    return hipGetLastError() == hipSuccess ? PTFLASH_OK : PTFLASH_EHIP;
}

// Compile-time dispatch over the component count.
template <template <int> class F, int NC = kMinNc>
struct Dispatch {
    template <typename... Args>
    static int run(int nc, Args &&...args)
    {
        if (nc == NC) return F<NC>::run(args...);
        if constexpr (NC < kMaxNc) return Dispatch<F, NC + 1>::run(nc, args...);
        return PTFLASH_EUNSUPPORTED;
    }
};

template <int NC>
struct PersistentF {
    static int run(const FlashArgs &a, const ptflash_problem *p, const ptflash_options *o,
                   void *ws, hipStream_t s)
    {
        return launch_persistent<NC>(a, p, o, ws, s);
    }
};

template <int NC>
struct PlainF {
    static int run(const FlashArgs &a, const ptflash_problem *p, void *ws, hipStream_t s)
    {
        return launch_plain<NC>(a, p, ws, s);
    }
};

template <int NC>
struct WsF {
    static int run(int64_t n, int form, size_t *out)
    {
        *out = workspace_bytes<NC>(n, form);
        return PTFLASH_OK;
    }
};

template <int NC>
struct BackwardF {
    static int run(const BwdArgs &b, const ptflash_problem *p, hipStream_t s)
    {
        const unsigned nb = (unsigned)((p->n + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(flash_backward_kernel<NC>, dim3(nb), dim3(kBlock), 0, s, b, p->Tc,
                           p->Pc, p->omega, p->kij);
        return hipGetLastError() == hipSuccess ? PTFLASH_OK : PTFLASH_EHIP;
    }
};

template <int NC>
struct EvalF {
    static int run(int64_t n, const double *c, const double *T, const double *P,
                   const double *Tc, const double *Pc, const double *om, const double *K,
                   double *lnphi, double *Z, double *phi, hipStream_t s)
    {
        return launch_eval<NC>(n, c, T, P, Tc, Pc, om, K, lnphi, Z, phi, s);
    }
};

static bool problem_ok(const ptflash_problem *p)
{
    if (!p || p->n < 0) return false;
    if (p->n == 0) return true;
    return p->z && p->T && p->P && p->Tc && p->Pc && p->omega && p->kij;
}

static bool options_ok(const ptflash_options *o)
{
    return o && o->max_pre_ss >= 1 && o->max_ss >= 0 && o->max_tr_sa >= 0 &&
           o->max_tr_split >= 0 && o->max_polish >= 0 && o->dem_every >= 0 &&
           o->tol_sa_ss > 0 && o->tol_sa_tr > 0 && o->tol_split_ss > 0 && o->tol_split_tr > 0 &&
           o->tol_polish > 0 && o->eps_tm >= 0 &&
           (o->form == PTFLASH_FORM_PERSISTENT || o->form == PTFLASH_FORM_PLAIN);
}

}  // namespace ptf

using namespace ptf;

extern "C" {

void ptflash_default_options(ptflash_options *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->max_pre_ss = 3;
    o->max_ss = 9;
    o->max_tr_sa = 20;
    o->max_tr_split = 20;
    o->max_polish = 4;
    o->dem_every = 5;
    o->tol_sa_ss = 1e-6;
    o->tol_sa_tr = 1e-6;
    o->tol_split_ss = 1e-8;
    o->tol_split_tr = 1e-8;
    o->tol_polish = 1e-13;
    o->eps_tm = 1e-10;
    o->form = PTFLASH_FORM_PERSISTENT;
    o->keep_factor = 0;
    o->block = 0;
    o->grid = 0;
}

int32_t ptflash_max_nc(void) { return kMaxNc; }

size_t ptflash_workspace_bytes(const ptflash_problem *p, const ptflash_options *o)
{
    if (!problem_ok(p) || !o) return 0;
    size_t b = 0;
    if (Dispatch<WsF>::run(p->nc, p->n, o->form, &b) != PTFLASH_OK) return 0;
    return b;
}

int ptflash_flash(const ptflash_problem *p, const ptflash_options *o, ptflash_result *r,
                  void *ws, size_t ws_bytes, hipStream_t s)
{
    if (!problem_ok(p) || !options_ok(o) || !r) return PTFLASH_EINVAL;
    if (p->nc < kMinNc || p->nc > kMaxNc) return PTFLASH_EUNSUPPORTED;
    if (p->props_per_mixture != 0) return PTFLASH_EUNSUPPORTED;
    if (p->n == 0) return PTFLASH_OK;
    if (p->n > (int64_t)1 << 30) return PTFLASH_EUNSUPPORTED;   // trial ids are 2m + t in 32 bits
    if (!r->label || !r->beta || !r->x || !r->y) return PTFLASH_EINVAL;
    if (o->keep_factor && !r->factor) return PTFLASH_EINVAL;
    if (!ws || ws_bytes < ptflash_workspace_bytes(p, o)) return PTFLASH_EWORKSPACE;
    if (((uintptr_t)ws & 255u) != 0) return PTFLASH_EINVAL;
    FlashArgs a;
    fill_args(a, p, o, r);
    if (o->form == PTFLASH_FORM_PLAIN) return Dispatch<PlainF>::run(p->nc, a, p, ws, s);
    return Dispatch<PersistentF>::run(p->nc, a, p, o, ws, s);
}

int ptflash_eval_phase(int64_t n, int32_t nc, const double *c, const double *T,
                       const double *P, const double *Tc, const double *Pc,
                       const double *omega, const double *kij, double *lnphi, double *Z,
                       double *phi, hipStream_t s)
{
    if (n < 0) return PTFLASH_EINVAL;
    if (nc < kMinNc || nc > kMaxNc) return PTFLASH_EUNSUPPORTED;
    if (n == 0) return PTFLASH_OK;
    if (!c || !T || !P || !Tc || !Pc || !omega || !kij || !lnphi || !Z) return PTFLASH_EINVAL;
    return Dispatch<EvalF>::run(nc, n, c, T, P, Tc, Pc, omega, kij, lnphi, Z, phi, s);
}

size_t ptflash_backward_workspace_bytes(const ptflash_problem *p, int32_t kij_reduce)
{
    if (!problem_ok(p)) return 0;
    const int64_t npair = (int64_t)p->nc * (p->nc - 1) / 2;
    if (kij_reduce) return 256 + align256((size_t)npair * (size_t)p->n * sizeof(double));
    return 256;
}

int ptflash_flash_backward(const ptflash_problem *p, const ptflash_options *o,
                           const ptflash_result *fwd, const double *g_beta, const double *g_x,
                           const double *g_y, double *g_z, double *g_T, double *g_P,
                           double *g_kij, int32_t kij_reduce, void *ws, size_t ws_bytes,
                           hipStream_t s)
{
    (void)o;
    if (!problem_ok(p) || !fwd) return PTFLASH_EINVAL;
    if (p->nc < kMinNc || p->nc > kMaxNc) return PTFLASH_EUNSUPPORTED;
    if (p->props_per_mixture != 0) return PTFLASH_EUNSUPPORTED;
    if (p->n == 0) return PTFLASH_OK;
    if (!fwd->label || !fwd->beta || !fwd->x || !fwd->y || !fwd->factor) return PTFLASH_EINVAL;
    if (!g_beta || !g_x || !g_y || !g_z || !g_T || !g_P || !g_kij) return PTFLASH_EINVAL;
    if (kij_reduce != 0 && kij_reduce != 1) return PTFLASH_EINVAL;
    const size_t need = ptflash_backward_workspace_bytes(p, kij_reduce);
    if (ws_bytes < need || (need > 0 && !ws)) return PTFLASH_EWORKSPACE;
    if (((uintptr_t)ws & 255u) != 0) return PTFLASH_EINVAL;
    BwdArgs b;
    b.n = p->n;
    b.z = p->z;
    b.T = p->T;
    b.P = p->P;
    b.label = fwd->label;
    b.beta = fwd->beta;
    b.x = fwd->x;
    b.y = fwd->y;
    b.factor = fwd->factor;
    b.status = fwd->status;
    b.gb = g_beta;
    b.gx = g_x;
    b.gy = g_y;
    b.gz = g_z;
    b.gT = g_T;
    b.gP = g_P;
    b.gk = kij_reduce ? nullptr : g_kij;
    b.kpart = kij_reduce ? (double *)((char *)ws + 256) : nullptr;
    int rc = Dispatch<BackwardF>::run(p->nc, b, p, s);
    if (rc) return rc;
    if (kij_reduce) {
        const int npair = p->nc * (p->nc - 1) / 2;
        hipLaunchKernelGGL(reduce_pairs, dim3(npair), dim3(kBlock), 0, s, b.kpart, p->n, p->nc,
                           g_kij);
        if (hipGetLastError() != hipSuccess) return PTFLASH_EHIP;
    }
    return PTFLASH_OK;
}

const char *ptflash_strerror(int code)
{
    switch (code) {
    case PTFLASH_OK: return "ok";
    case PTFLASH_EINVAL: return "invalid argument";
    case PTFLASH_EUNSUPPORTED: return "unsupported component count, layout or form";
    case PTFLASH_EWORKSPACE: return "workspace too small";
    case PTFLASH_EHIP: return "HIP runtime error";
    default: return "unknown error";
    }
}

}  // extern "C"
