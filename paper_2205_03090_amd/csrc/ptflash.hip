// ptflash.hip -- C ABI of the gfx950 SRK PT flash: argument checks,
// workspace sizes and the dispatch over the component count to the per-nc
// launchers (flash_nc.hip, compiled once per nc), plus the batch reduction of
// the k gradient.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "ptflash.h"
#include "flash_api.hpp"

namespace ptf {

constexpr int kBlock = 256;

// Deterministic batch sum of the k contributions in two passes.  Pass 1:
// block (q, c) sums mixtures [c*kRedChunk, (c+1)*kRedChunk) of pair q (each
// thread a fixed strided subset in order, then a fixed tree in LDS).  Pass
// 2: one block per pair sums its chunk partials the same way.  The order of
// every addition is fixed by n alone, so the result does not depend on
// scheduling.
constexpr int64_t kRedChunk = 16384;

__device__ __forceinline__ double block_tree_sum(double v, double *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    return red[0];
}

__global__ void __launch_bounds__(kBlock)
reduce_pairs_chunks(const double *__restrict__ kpart, int64_t n, int64_t nchunk, double *part)
{
    __shared__ double red[kBlock];
    const int64_t q = blockIdx.y, c = blockIdx.x;
    const int64_t lo = c * kRedChunk, hi = lo + kRedChunk < n ? lo + kRedChunk : n;
    double acc = 0.0;
    for (int64_t m = lo + threadIdx.x; m < hi; m += kBlock) acc += kpart[q * n + m];
    const double t = block_tree_sum(acc, red);
    if (threadIdx.x == 0) part[q * nchunk + c] = t;
}

__global__ void __launch_bounds__(kBlock)
reduce_pairs_final(const double *__restrict__ part, int64_t nchunk, int nc, double *gk)
{
    __shared__ double red[kBlock];
    const int q = blockIdx.x;
    double acc = 0.0;
    for (int64_t c = threadIdx.x; c < nchunk; c += kBlock) acc += part[(int64_t)q * nchunk + c];
    const double t = block_tree_sum(acc, red);
    if (threadIdx.x == 0) {
        // pair index -> (i, j), i < j
        int i = 0, r = q;
        while (r >= nc - 1 - i) { r -= nc - 1 - i; ++i; }
        const int j = i + 1 + r;
        gk[i * nc + j] = 0.5 * t;
        gk[j * nc + i] = 0.5 * t;
        if (q == 0)
            for (int d = 0; d < nc; ++d) gk[d * nc + d] = 0.0;
    }
}

static int64_t red_chunks(int64_t n) { return (n + kRedChunk - 1) / kRedChunk; }

// Workspace of ptflash_flash_noalloc: a static device array (one copy on
// every GPU the library runs on, kept until the process ends).  Its name is
// a host-side stand-in; the device address comes from hipGetSymbolAddress,
// looked up once per device (with that device current) and kept here.
constexpr size_t kScratchBytes = PTFLASH_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_addr[kMaxDevices] = {};

static int scratch_address(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return PTFLASH_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return PTFLASH_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *a = nullptr;
        if (hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)) != hipSuccess || !a) return PTFLASH_EHIP;
        g_scratch_addr[dev] = a;
    }
    *out = g_scratch_addr[dev];
    return PTFLASH_OK;
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
    a.tm = r->tm;
    a.stability_only = 0;
    a.lnk0 = p->lnk0;
    a.hint = p->hint;
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
struct FlashF {
    static int run(const FlashArgs &a, const ptflash_problem *p, const ptflash_options *o,
                   void *ws, hipStream_t s)
    {
        return p->props_per_mixture ? nc_flash_pm<NC, true>(a, p, o, ws, s)
                                    : nc_flash_pm<NC, false>(a, p, o, ws, s);
    }
};

template <int NC>
struct WsF {
    static int run(int64_t n, int form, size_t *out)
    {
        *out = nc_workspace_bytes<NC>(n, form);
        return PTFLASH_OK;
    }
};

template <int NC>
struct BackwardF {
    static int run(const BwdArgs &b, const ptflash_problem *p, hipStream_t s)
    {
        return p->props_per_mixture ? nc_backward_pm<NC, true>(b, p, s)
                                    : nc_backward_pm<NC, false>(b, p, s);
    }
};

template <int NC>
struct EvalF {
    static int run(int64_t n, const double *c, const double *T, const double *P,
                   const double *Tc, const double *Pc, const double *om, const double *K,
                   double *lnphi, double *Z, double *phi, hipStream_t s)
    {
        return nc_eval<NC>(n, c, T, P, Tc, Pc, om, K, lnphi, Z, phi, s);
    }
};

// ---------------------------------------------------------------------------
// Ragged batches: grouping by nc, gather into uniform batches, scatter back
// ---------------------------------------------------------------------------

constexpr int kBuckets = 32;   // bucket 0: invalid; 2..kMaxNc: by nc
static_assert(kMaxNc < kBuckets, "bucket table too small");

__device__ __forceinline__ int ragged_bucket(int64_t m, const int32_t *nc_of, const int64_t *off)
{
    const int nc = nc_of[m];
    if (nc < kMinNc || nc > kMaxNc) return 0;
    if (off[m + 1] - off[m] != (int64_t)nc) return 0;
    return nc;
}

__global__ void __launch_bounds__(kBlock)
ragged_count(int64_t n, const int32_t *__restrict__ nc_of, const int64_t *__restrict__ off,
             unsigned long long *counts)
{
    __shared__ unsigned int h[kBuckets];
    if (threadIdx.x < kBuckets) h[threadIdx.x] = 0u;
    __syncthreads();
    for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < n;
         m += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&h[ragged_bucket(m, nc_of, off)], 1u);
    __syncthreads();
    if (threadIdx.x < kBuckets && h[threadIdx.x] > 0u)
        atomicAdd(&counts[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

struct BucketStarts {
    int64_t s[kBuckets];
};

// Counting sort of the mixture ids by bucket (the order inside a bucket is
// arbitrary; every mixture's result depends on its own data only).  Ranks
// inside a block come from LDS atomics; each block then claims its range of
// every bucket with one device atomic (per-mixture device atomics on the
// few bucket counters serialise).
__global__ void __launch_bounds__(kBlock)
ragged_sort(int64_t n, const int32_t *__restrict__ nc_of, const int64_t *__restrict__ off,
            BucketStarts st, unsigned long long *cursor, uint32_t *ids)
{
    __shared__ unsigned int cnt[kBuckets];
    __shared__ unsigned long long base[kBuckets];
    if (threadIdx.x < kBuckets) cnt[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int b = m < n ? ragged_bucket(m, nc_of, off) : 0;
    const unsigned int r = m < n ? atomicAdd(&cnt[b], 1u) : 0u;
    __syncthreads();
    if (threadIdx.x < kBuckets && cnt[threadIdx.x] > 0u)
        base[threadIdx.x] = atomicAdd(&cursor[threadIdx.x], (unsigned long long)cnt[threadIdx.x]);
    __syncthreads();
    if (m < n) ids[st.s[b] + (int64_t)(base[b] + r)] = (uint32_t)m;
}

struct RaggedIn {
    const int64_t *off, *koff;
    const double *z, *T, *P, *Tc, *Pc, *om, *K;
    const double *lnk0;   // optional warm-start inputs (null: none)
    const int8_t *hint;
};

struct Uniform {   // one gathered uniform-nc chunk
    double *z, *T, *P, *Tc, *Pc, *om, *K, *lnk0;
    int8_t *hint;
    int8_t *label;
    double *beta, *x, *y, *tm;
    int16_t *iters;
    uint16_t *status;
    uint32_t *flops;
};

// Gather of one uniform chunk, one thread per value (coalesced stores, and
// loads that walk each mixture's contiguous rows): the per-component rows
// (z, Tc, Pc, omega and the optional initial ln K; T, P and the optional
// hint with component 0) ...
template <int NC>
__global__ void __launch_bounds__(kBlock)
ragged_gather_rows(int64_t cnt, const uint32_t *__restrict__ ids, RaggedIn in, Uniform u)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt * NC) return;
    const int64_t j = t / NC;
    const int e = (int)(t - j * NC);
    const int64_t m = ids[j];
    const int64_t o = in.off[m] + e;
    u.z[t] = in.z[o];
    u.Tc[t] = in.Tc[o];
    u.Pc[t] = in.Pc[o];
    u.om[t] = in.om[o];
    if (in.lnk0) u.lnk0[t] = in.lnk0[o];
    if (e == 0) {
        u.T[j] = in.T[m];
        u.P[j] = in.P[m];
        if (in.hint) u.hint[j] = in.hint[m];
    }
}

// ... and the k blocks.
template <int NC>
__global__ void __launch_bounds__(kBlock)
ragged_gather_k(int64_t cnt, const uint32_t *__restrict__ ids, RaggedIn in, Uniform u)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt * NC * NC) return;
    const int64_t j = t / (NC * NC);
    const int e = (int)(t - j * (NC * NC));
    u.K[t] = in.K[in.koff[ids[j]] + e];
}

// Scatter of one chunk's outputs, one thread per x/y value (per-mixture
// fields with component 0).
template <int NC>
__global__ void __launch_bounds__(kBlock)
ragged_scatter_rows(int64_t cnt, const uint32_t *__restrict__ ids, const int64_t *off, Uniform u,
                    ptflash_result r)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt * NC) return;
    const int64_t j = t / NC;
    const int e = (int)(t - j * NC);
    const int64_t m = ids[j];
    const int64_t o = off[m] + e;
    r.x[o] = u.x[t];
    r.y[o] = u.y[t];
    if (e == 0) {
        r.label[m] = u.label[j];
        r.beta[m] = u.beta[j];
        if (r.iters)
            for (int k = 0; k < PTFLASH_NITERS; ++k)
                r.iters[m * PTFLASH_NITERS + k] = u.iters[j * PTFLASH_NITERS + k];
        if (r.status) r.status[m] = u.status[j];
        if (r.flops) r.flops[m] = u.flops[j];
        if (r.tm) r.tm[m] = u.tm[j];
    }
}

template <int NC>
void ragged_move(bool gather, int64_t cnt, const uint32_t *ids, const RaggedIn &in,
                 const Uniform &u, const int64_t *off, const ptflash_result &r, hipStream_t s)
{
    auto grid = [](int64_t k) { return dim3((unsigned)((k + kBlock - 1) / kBlock)); };
    if (gather) {
        hipLaunchKernelGGL(ragged_gather_rows<NC>, grid(cnt * NC), dim3(kBlock), 0, s, cnt, ids,
                           in, u);
        hipLaunchKernelGGL(ragged_gather_k<NC>, grid(cnt * NC * NC), dim3(kBlock), 0, s, cnt,
                           ids, in, u);
    } else {
        hipLaunchKernelGGL(ragged_scatter_rows<NC>, grid(cnt * NC), dim3(kBlock), 0, s, cnt,
                           ids, off, u, r);
    }
}

template <int NC>
struct RaggedMove {
    static void run(int nc, bool gather, int64_t cnt, const uint32_t *ids, const RaggedIn &in,
                    const Uniform &u, const int64_t *off, const ptflash_result &r, hipStream_t s)
    {
        if (nc == NC) ragged_move<NC>(gather, cnt, ids, in, u, off, r, s);
        else if constexpr (NC < kMaxNc) RaggedMove<NC + 1>::run(nc, gather, cnt, ids, in, u, off, r, s);
    }
};

// Mixtures whose nc or row count is unusable: single phase, INVALID, with
// the raw z rows they do have copied to x and y.
__global__ void __launch_bounds__(kBlock)
ragged_invalid(int64_t cnt, const uint32_t *__restrict__ ids, const int64_t *off,
               const double *z, ptflash_result r)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cnt) return;
    const int64_t m = ids[j];
    r.label[m] = 0;
    r.beta[m] = -1.0;
    for (int64_t i = off[m]; i < off[m + 1]; ++i) {
        r.x[i] = z[i];
        r.y[i] = z[i];
    }
    if (r.iters)
        for (int k = 0; k < PTFLASH_NITERS; ++k) r.iters[m * PTFLASH_NITERS + k] = 0;
    if (r.status) r.status[m] = (uint16_t)PTFLASH_ST_INVALID;
    if (r.flops) r.flops[m] = 0u;
    if (r.tm) r.tm[m] = NAN;
}

__global__ void zero_u64(unsigned long long *q, int n)
{
    if ((int)threadIdx.x < n) q[threadIdx.x] = 0ull;
}

// Largest number of mixtures gathered and flashed at once.
static int64_t ragged_chunk(int64_t n, int form)
{
    const int64_t cap = form == PTFLASH_FORM_PLAIN ? ((int64_t)1 << 18) : ((int64_t)1 << 20);
    return n < cap ? n : cap;
}

// Ragged workspace: counters | sorted ids | one uniform chunk (inputs,
// outputs) | the uniform flash's workspace for that chunk at nc = kMaxNc.
static size_t ragged_ws_layout(int64_t n, int form, size_t *flash_off)
{
    const size_t ch = (size_t)ragged_chunk(n, form), C = (size_t)kMaxNc;
    size_t b = align256(2 * kBuckets * sizeof(unsigned long long));
    b += align256((size_t)n * 4);
    b += align256(ch * C * 8) * 6 + align256(ch * C * C * 8) + align256(ch * 8) * 3 +
         align256(ch) + align256(ch * PTFLASH_NITERS * 2) + align256(ch * 2) + align256(ch * 4) +
         align256(ch * 8) + align256(ch * C * 8) + align256(ch);
    *flash_off = b;
    size_t fw = 0;
    if (Dispatch<WsF>::run(kMaxNc, (int64_t)ch, form, &fw) != PTFLASH_OK) return 0;
    return b + fw;
}

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
           (o->form == PTFLASH_FORM_PERSISTENT || o->form == PTFLASH_FORM_PLAIN ||
            o->form == PTFLASH_FORM_FUSED) &&
           (o->lanes_per_mixture == 0 || o->lanes_per_mixture == 1 ||
            o->lanes_per_mixture == 16 || o->lanes_per_mixture == 32) &&
           (o->lanes_split == 0 || o->lanes_split == 1 || o->lanes_split == 16 ||
            o->lanes_split == 32) &&
           (o->lanes_ss == 0 || o->lanes_ss == 1 || o->lanes_ss == 16 || o->lanes_ss == 32);
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
    o->max_tr_split = 30;
    o->max_polish = 4;
    o->dem_every = 3;
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
    o->lanes_per_mixture = 0;
    o->lanes_split = 0;
    o->lanes_ss = 0;
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
    if (p->props_per_mixture != 0 && p->props_per_mixture != 1) return PTFLASH_EINVAL;
    if (p->n == 0) return PTFLASH_OK;
    if (p->n > (int64_t)1 << 30) return PTFLASH_EUNSUPPORTED;   // trial ids are 2m + t in 32 bits
    if (!r->label || !r->beta || !r->x || !r->y) return PTFLASH_EINVAL;
    if (o->keep_factor && !r->factor) return PTFLASH_EINVAL;
    if (!ws || ws_bytes < ptflash_workspace_bytes(p, o)) return PTFLASH_EWORKSPACE;
    if (((uintptr_t)ws & 255u) != 0) return PTFLASH_EINVAL;
    FlashArgs a;
    fill_args(a, p, o, r);
    return Dispatch<FlashF>::run(p->nc, a, p, o, ws, s);
}

int ptflash_stability(const ptflash_problem *p, const ptflash_options *o, ptflash_result *r,
                      void *ws, size_t ws_bytes, hipStream_t s)
{
    if (!problem_ok(p) || !options_ok(o) || !r) return PTFLASH_EINVAL;
    if (p->nc < kMinNc || p->nc > kMaxNc) return PTFLASH_EUNSUPPORTED;
    if (p->props_per_mixture != 0 && p->props_per_mixture != 1) return PTFLASH_EINVAL;
    if (p->n == 0) return PTFLASH_OK;
    if (p->n > (int64_t)1 << 30) return PTFLASH_EUNSUPPORTED;
    if (!r->label || o->keep_factor) return PTFLASH_EINVAL;
    if (!ws || ws_bytes < ptflash_workspace_bytes(p, o)) return PTFLASH_EWORKSPACE;
    if (((uintptr_t)ws & 255u) != 0) return PTFLASH_EINVAL;
    FlashArgs a;
    fill_args(a, p, o, r);
    a.beta = nullptr;
    a.x = nullptr;
    a.y = nullptr;
    a.factor = nullptr;
    a.stability_only = 1;
    return Dispatch<FlashF>::run(p->nc, a, p, o, ws, s);
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
    if (kij_reduce)
        return 256 + align256((size_t)npair * (size_t)p->n * sizeof(double)) +
               align256((size_t)npair * (size_t)red_chunks(p->n) * sizeof(double));
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
    if (p->props_per_mixture != 0 && p->props_per_mixture != 1) return PTFLASH_EINVAL;
    if (p->props_per_mixture && kij_reduce) return PTFLASH_EINVAL;
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
        const int64_t nch = red_chunks(p->n);
        double *part = b.kpart + align256((size_t)npair * (size_t)p->n * sizeof(double)) / 8;
        hipLaunchKernelGGL(reduce_pairs_chunks, dim3((unsigned)nch, (unsigned)npair), dim3(kBlock),
                           0, s, b.kpart, p->n, nch, part);
        hipLaunchKernelGGL(reduce_pairs_final, dim3(npair), dim3(kBlock), 0, s, part, nch, p->nc,
                           g_kij);
        if (hipGetLastError() != hipSuccess) return PTFLASH_EHIP;
    }
    return PTFLASH_OK;
}

size_t ptflash_ragged_workspace_bytes(const ptflash_ragged_problem *p,
                                      const ptflash_options *o)
{
    if (!p || !o || p->n < 0) return 0;
    size_t fo = 0;
    return ragged_ws_layout(p->n, o->form, &fo);
}

int ptflash_flash_ragged(const ptflash_ragged_problem *p, const ptflash_options *o,
                         ptflash_result *r, void *ws, size_t ws_bytes, hipStream_t s)
{
    if (!p || p->n < 0 || !options_ok(o) || !r) return PTFLASH_EINVAL;
    if (p->n == 0) return PTFLASH_OK;
    if (p->n > (int64_t)1 << 30) return PTFLASH_EUNSUPPORTED;
    if (!p->nc_of || !p->off || !p->koff || !p->z || !p->T || !p->P || !p->Tc || !p->Pc ||
        !p->omega || !p->kij)
        return PTFLASH_EINVAL;
    if (!r->label || !r->beta || !r->x || !r->y) return PTFLASH_EINVAL;
    if (o->keep_factor || r->factor) return PTFLASH_EINVAL;
    size_t foff = 0;
    const size_t need = ragged_ws_layout(p->n, o->form, &foff);
    if (!ws || need == 0 || ws_bytes < need) return PTFLASH_EWORKSPACE;
    if (((uintptr_t)ws & 255u) != 0) return PTFLASH_EINVAL;
    const int64_t n = p->n, ch = ragged_chunk(n, o->form), C = kMaxNc;
    char *w = (char *)ws;
    unsigned long long *counts = (unsigned long long *)w;
    unsigned long long *cursor = counts + kBuckets;
    w += align256(2 * kBuckets * sizeof(unsigned long long));
    uint32_t *ids = (uint32_t *)w;
    w += align256((size_t)n * 4);
    Uniform u;
    auto takeb = [&](size_t bytes) { char *q = w; w += align256(bytes); return q; };
    u.z = (double *)takeb(ch * C * 8);
    u.Tc = (double *)takeb(ch * C * 8);
    u.Pc = (double *)takeb(ch * C * 8);
    u.om = (double *)takeb(ch * C * 8);
    u.x = (double *)takeb(ch * C * 8);
    u.y = (double *)takeb(ch * C * 8);
    u.K = (double *)takeb(ch * C * C * 8);
    u.T = (double *)takeb(ch * 8);
    u.P = (double *)takeb(ch * 8);
    u.beta = (double *)takeb(ch * 8);
    u.label = (int8_t *)takeb(ch);
    u.iters = (int16_t *)takeb(ch * PTFLASH_NITERS * 2);
    u.status = (uint16_t *)takeb(ch * 2);
    u.flops = (uint32_t *)takeb(ch * 4);
    u.tm = (double *)takeb(ch * 8);
    u.lnk0 = (double *)takeb(ch * C * 8);
    u.hint = (int8_t *)takeb(ch);
    void *fws = (char *)ws + foff;
    const size_t fws_bytes = ws_bytes - foff;

    // group sizes (one host synchronisation)
    hipLaunchKernelGGL(zero_u64, dim3(1), dim3(64), 0, s, counts, 2 * kBuckets);
    const int64_t blocks = (n + kBlock - 1) / kBlock;
    const unsigned cgrid = (unsigned)(blocks < 4096 ? blocks : 4096);
    hipLaunchKernelGGL(ragged_count, dim3(cgrid), dim3(kBlock), 0, s, n, p->nc_of, p->off,
                       counts);
    unsigned long long hc[kBuckets];
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(hc, counts, sizeof(hc), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return PTFLASH_EHIP;
    BucketStarts st;
    int64_t acc = 0;
    for (int b = 0; b < kBuckets; ++b) { st.s[b] = acc; acc += (int64_t)hc[b]; }
    hipLaunchKernelGGL(ragged_sort, dim3((unsigned)blocks), dim3(kBlock), 0, s, n, p->nc_of,
                       p->off, st, cursor, ids);
    ptflash_result rr = *r;
    if (hc[0] > 0)
        hipLaunchKernelGGL(ragged_invalid, dim3((unsigned)((hc[0] + kBlock - 1) / kBlock)),
                           dim3(kBlock), 0, s, (int64_t)hc[0], ids, p->off, p->z, rr);
    if (hipGetLastError() != hipSuccess) return PTFLASH_EHIP;
    const RaggedIn in{p->off, p->koff, p->z, p->T, p->P, p->Tc, p->Pc, p->omega, p->kij,
                      p->lnk0, p->hint};
    for (int nc = kMinNc; nc <= kMaxNc; ++nc) {
        for (int64_t c0 = 0; c0 < (int64_t)hc[nc]; c0 += ch) {
            const int64_t cnt = ((int64_t)hc[nc] - c0) < ch ? ((int64_t)hc[nc] - c0) : ch;
            const uint32_t *cid = ids + st.s[nc] + c0;
            RaggedMove<kMinNc>::run(nc, true, cnt, cid, in, u, p->off, rr, s);
            ptflash_problem sub{cnt, nc, 1, u.z, u.T, u.P, u.Tc, u.Pc, u.om, u.K,
                                p->lnk0 ? u.lnk0 : nullptr, p->hint ? u.hint : nullptr};
            ptflash_result sr{u.label, u.beta, u.x, u.y, u.iters, u.status, u.flops, nullptr,
                              r->tm ? u.tm : nullptr};
            if (fws_bytes < ptflash_workspace_bytes(&sub, o)) return PTFLASH_EWORKSPACE;
            FlashArgs a;
            fill_args(a, &sub, o, &sr);
            int rc = Dispatch<FlashF>::run(nc, a, &sub, o, fws, s);
            if (rc) return rc;
            RaggedMove<kMinNc>::run(nc, false, cnt, cid, in, u, p->off, rr, s);
            if (hipGetLastError() != hipSuccess) return PTFLASH_EHIP;
        }
    }
    return PTFLASH_OK;
}

int ptflash_flash_noalloc(const ptflash_problem *p, const ptflash_options *o,
                          ptflash_result *r, hipStream_t s)
{
    if (!problem_ok(p) || !options_ok(o) || !r) return PTFLASH_EINVAL;
    if (p->nc < kMinNc || p->nc > kMaxNc) return PTFLASH_EUNSUPPORTED;
    if (p->n == 0) return PTFLASH_OK;
    if (ptflash_workspace_bytes(p, o) > kScratchBytes) return PTFLASH_EWORKSPACE;
    void *ws = nullptr;
    const int rc = scratch_address(&ws);
    if (rc != PTFLASH_OK) return rc;
    return ptflash_flash(p, o, r, ws, kScratchBytes, s);
}

const char *ptflash_strerror(int code)
{
    switch (code) {
    case PTFLASH_OK: return "ok";
    case PTFLASH_EINVAL: return "invalid argument";
    case PTFLASH_EUNSUPPORTED: return "unsupported component count, layout or form";
    case PTFLASH_EWORKSPACE:
        return "workspace too small (ptflash_flash_noalloc: problem exceeds its scratch buffer)";
    case PTFLASH_EHIP: return "HIP runtime error";
    default: return "unknown error";
    }
}

}  // extern "C"
