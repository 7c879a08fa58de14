// ptflash.hip -- kernels and C ABI of the gfx950 SRK PT flash.
//
// Persistent form: a grid sized to the device; every wavefront keeps one
// mixture per lane and, whenever lanes finish, takes the next mixture
// indices from a device counter (one atomic per wavefront and step), so
// converged mixtures leave the wave immediately and their lanes are reused.
// This is the paper's "synchronizer" (save converged rows, drop them from
// the active set; Sec. 3, Algorithm 1) done per lane inside one launch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "ptflash.h"
#include "flash_lane.hpp"
#include "adjoint_device.hpp"

namespace ptf {

constexpr int kMinNc = 2;
constexpr int kMaxNc = PTF_MAX_NC;
constexpr int kBlock = 256;

__global__ void reset_counter(unsigned long long *q) { *q = 0ull; }

template <int NC>
__global__ void __launch_bounds__(kBlock)
flash_persistent(FlashArgs a, const double *__restrict__ Tc, const double *__restrict__ Pc,
                 const double *__restrict__ om, const double *__restrict__ K,
                 unsigned long long *__restrict__ queue)
{
    const Props pr{Tc, Pc, om, K};
    Lane<NC> L;
    L.stage = ST_IDLE;
    const int lane = (int)__lane_id();
    for (;;) {
        const bool want = (L.stage == ST_IDLE);
        const unsigned long long mask = __ballot(want);
        if (mask) {
            const int leader = __ffsll((unsigned long long)mask) - 1;
            unsigned long long base = 0;
            if (lane == leader) base = atomicAdd(queue, (unsigned long long)__popcll(mask));
            const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)base, leader);
            const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(base >> 32), leader);
            base = ((unsigned long long)hi << 32) | lo;
            if (want) {
                const unsigned long long below = mask & ((1ull << lane) - 1ull);
                const long long mi = (long long)(base + (unsigned long long)__popcll(below));
                if (mi < a.n) L.start(mi, a, pr);
                else L.stage = ST_GONE;
            }
        }
        if (__ballot(L.stage != ST_GONE) == 0ull) break;
        L.step(a, pr);
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
// Plain form: the paper's synchronizer with a barrier per stage (Sec. 3,
// Algorithm 1).  Per-mixture state lives in global memory; each launch
// advances every mixture of the current stage by one step; a compaction
// kernel then lists the mixtures still in that stage and the host reads the
// count.  Stages run in order, so a stage starts only when the previous one
// has no mixture left.  The per-mixture arithmetic is Lane::step(), the same
// as in the persistent form.
// ---------------------------------------------------------------------------

template <int NC>
__global__ void __launch_bounds__(kBlock)
plain_init(FlashArgs a, const double *__restrict__ Tc, const double *__restrict__ Pc,
           const double *__restrict__ om, const double *__restrict__ K, Lane<NC> *states,
           int32_t *list, unsigned long long *count)
{
    const Props pr{Tc, Pc, om, K};
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= a.n) return;
    Lane<NC> L;
    L.start(m, a, pr);
    states[m] = L;
    if (L.stage == ST_FEED) {
        const unsigned long long k = atomicAdd(count, 1ull);
        list[k] = (int32_t)m;
    }
}

template <int NC>
__global__ void __launch_bounds__(kBlock)
plain_step(FlashArgs a, const double *__restrict__ Tc, const double *__restrict__ Pc,
           const double *__restrict__ om, const double *__restrict__ K, Lane<NC> *states,
           const int32_t *__restrict__ list, int64_t count)
{
    const Props pr{Tc, Pc, om, K};
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const int32_t m = list[k];
    Lane<NC> L = states[m];
    L.step(a, pr);
    states[m] = L;
}

// Lists the mixtures of `in` whose stage equals (keep_equal = 1) or differs
// from (keep_equal = 0) `stage`; the order is not deterministic, which does
// not matter since each mixture's result depends on its own state only.
template <int NC>
__global__ void __launch_bounds__(kBlock)
plain_compact(const Lane<NC> *__restrict__ states, const int32_t *__restrict__ in,
              int64_t count, int stage, int keep_equal, int32_t *out, unsigned long long *outc)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const int32_t m = in[k];
    if ((states[m].stage == stage) == (keep_equal != 0)) {
        const unsigned long long j = atomicAdd(outc, 1ull);
        out[j] = m;
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
    // every stage's evaluations are bounded by its caps (a rejected
    // trust-region step costs one extra evaluation); the cap below is a
    // safety net that guarantees termination
    a.max_steps = 8 + o->max_pre_ss + (o->max_ss + 2 + 2 * o->max_tr_sa) +
                  (o->max_ss + 2) + (2 * o->max_tr_split + o->max_polish + 4);
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

template <int NC>
static int launch_persistent(const FlashArgs &a, const ptflash_problem *p,
                             const ptflash_options *o, unsigned long long *queue,
                             hipStream_t s)
{
    const int block = o->block > 0 ? o->block : kBlock;
    if (block % 64 != 0 || block > kBlock) return PTFLASH_EINVAL;
    int grid = o->grid;
    if (grid <= 0) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, flash_persistent<NC>, block,
                                                         0) != hipSuccess)
            return PTFLASH_EHIP;
        const int cus = device_cus();
        if (cus <= 0) return PTFLASH_EHIP;
        grid = (per_cu > 0 ? per_cu : 1) * cus;
    }
    hipLaunchKernelGGL(reset_counter, dim3(1), dim3(1), 0, s, queue);
    hipLaunchKernelGGL(flash_persistent<NC>, dim3(grid), dim3(block), 0, s, a, p->Tc, p->Pc,
                       p->omega, p->kij, queue);
    return hipGetLastError() == hipSuccess ? PTFLASH_OK : PTFLASH_EHIP;
}

static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

template <int NC>
static size_t plain_workspace(int64_t n)
{
    return 256 + align256((size_t)n * sizeof(Lane<NC>)) + 3 * align256((size_t)n * sizeof(int32_t));
}

// Reads the device counter after the work queued so far (host sync).
static int read_count(unsigned long long *dcnt, int64_t &out, hipStream_t s)
{
    unsigned long long h = 0;
    if (hipGetLastError() != hipSuccess) return PTFLASH_EHIP;
    if (hipMemcpyAsync(&h, dcnt, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return PTFLASH_EHIP;
    out = (int64_t)h;
    return PTFLASH_OK;
}

template <int NC>
static int launch_plain(const FlashArgs &a, const ptflash_problem *p, void *ws, hipStream_t s)
{
    char *base = (char *)ws;
    unsigned long long *cnt = (unsigned long long *)base;
    const size_t st = align256((size_t)p->n * sizeof(Lane<NC>));
    const size_t li = align256((size_t)p->n * sizeof(int32_t));
    Lane<NC> *states = (Lane<NC> *)(base + 256);
    int32_t *live = (int32_t *)(base + 256 + st);
    int32_t *wa = (int32_t *)(base + 256 + st + li);
    int32_t *wb = (int32_t *)(base + 256 + st + 2 * li);
    auto grid = [](int64_t c) { return dim3((unsigned)((c + kBlock - 1) / kBlock)); };
    hipLaunchKernelGGL(reset_counter, dim3(1), dim3(1), 0, s, cnt);
    hipLaunchKernelGGL(plain_init<NC>, grid(p->n), dim3(kBlock), 0, s, a, p->Tc, p->Pc,
                       p->omega, p->kij, states, live, cnt);
    int64_t nlive = 0;
    int rc = read_count(cnt, nlive, s);
    if (rc) return rc;
    const int stages[5] = {ST_FEED, ST_PRE, ST_SA, ST_SPLIT_SS, ST_SPLIT_NT};
    for (int si = 0; si < 5 && nlive > 0; ++si) {
        const int stage = stages[si];
        // barrier: the stage starts with every live mixture that reached it
        int64_t nw = 0;
        hipLaunchKernelGGL(reset_counter, dim3(1), dim3(1), 0, s, cnt);
        hipLaunchKernelGGL(plain_compact<NC>, grid(nlive), dim3(kBlock), 0, s, states, live,
                           nlive, stage, 1, wa, cnt);
        if ((rc = read_count(cnt, nw, s))) return rc;
        int32_t *work = wa, *spare = wb;
        for (int guard = 0; nw > 0 && guard <= a.max_steps; ++guard) {
            hipLaunchKernelGGL(plain_step<NC>, grid(nw), dim3(kBlock), 0, s, a, p->Tc, p->Pc,
                               p->omega, p->kij, states, work, nw);
            hipLaunchKernelGGL(reset_counter, dim3(1), dim3(1), 0, s, cnt);
            hipLaunchKernelGGL(plain_compact<NC>, grid(nw), dim3(kBlock), 0, s, states, work, nw,
                               stage, 1, spare, cnt);
            if ((rc = read_count(cnt, nw, s))) return rc;
            int32_t *t = work; work = spare; spare = t;
        }
        // drop finished mixtures from the live list
        hipLaunchKernelGGL(reset_counter, dim3(1), dim3(1), 0, s, cnt);
        hipLaunchKernelGGL(plain_compact<NC>, grid(nlive), dim3(kBlock), 0, s, states, live,
                           nlive, (int)ST_IDLE, 0, wb, cnt);
        if ((rc = read_count(cnt, nlive, s))) return rc;
        if (nlive > 0 &&
            hipMemcpyAsync(live, wb, (size_t)nlive * sizeof(int32_t), hipMemcpyDeviceToDevice, s) !=
                hipSuccess)
            return PTFLASH_EHIP;
    }
    return hipGetLastError() == hipSuccess ? PTFLASH_OK : PTFLASH_EHIP;
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
                   unsigned long long *q, hipStream_t s)
    {
        return launch_persistent<NC>(a, p, o, q, s);
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
struct PlainWsF {
    static int run(int64_t n, size_t *out)
    {
        *out = plain_workspace<NC>(n);
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
    if (o->form == PTFLASH_FORM_PLAIN) {
        size_t b = 0;
        if (Dispatch<PlainWsF>::run(p->nc, p->n, &b) != PTFLASH_OK) return 0;
        return b;
    }
    return 256;
}

int ptflash_flash(const ptflash_problem *p, const ptflash_options *o, ptflash_result *r,
                  void *ws, size_t ws_bytes, hipStream_t s)
{
    if (!problem_ok(p) || !options_ok(o) || !r) return PTFLASH_EINVAL;
    if (p->nc < kMinNc || p->nc > kMaxNc) return PTFLASH_EUNSUPPORTED;
    if (p->props_per_mixture != 0) return PTFLASH_EUNSUPPORTED;
    if (p->n == 0) return PTFLASH_OK;
    if (o->form == PTFLASH_FORM_PLAIN && p->n > INT32_MAX) return PTFLASH_EUNSUPPORTED;
    if (!r->label || !r->beta || !r->x || !r->y) return PTFLASH_EINVAL;
    if (o->keep_factor && !r->factor) return PTFLASH_EINVAL;
    if (!ws || ws_bytes < ptflash_workspace_bytes(p, o)) return PTFLASH_EWORKSPACE;
    if (((uintptr_t)ws & 255u) != 0) return PTFLASH_EINVAL;
    FlashArgs a;
    fill_args(a, p, o, r);
    if (o->form == PTFLASH_FORM_PLAIN) return Dispatch<PlainF>::run(p->nc, a, p, ws, s);
    return Dispatch<PersistentF>::run(p->nc, a, p, o, (unsigned long long *)ws, s);
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
