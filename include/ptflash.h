/*
 * ptflash.h -- C ABI of the MI355X (gfx950) isothermal two-phase PT flash
 * with the Soave-Redlich-Kwong equation of state.
 *
 * The operation is the flash of Qu et al., "PTFlash" (arXiv 2205.03090):
 * given pressure P, temperature T and feed composition z of a mixture of nc
 * components (critical temperatures Tc, critical pressures Pc, acentric
 * factors omega, binary interaction parameters k_ij), decide whether the
 * mixture is a single phase or splits into two, and in the latter case return
 * the vapour fraction beta (theta_V) and the liquid and vapour compositions
 * x, y that satisfy the material balance and equal fugacities (Sec. 2.1,
 * eqs. material_balance and eq_cond).  Per mixture: Wilson K (eq. wilson),
 * three phase-split substitutions and the three-case triage (Sec. 2.2.3),
 * Michelsen stability analysis from a vapour-like and a liquid-like trial by
 * successive substitution with dominant-eigenvalue acceleration and a trust
 * region (Sec. 2.2.1, Appendix B.1), the K re-estimate, Rachford-Rice
 * (eq. RR, Appendix C), successive substitution of the phase split and a
 * trust-region Newton method on the reduced Gibbs energy (Sec. 2.2.2,
 * Appendix B.2), followed by Newton refinement of the converged split to
 * the double-precision root of the equal-fugacity system.
 *
 * Conventions shared by every entry point:
 *  - All array pointers are DEVICE pointers (HIP global memory), owned by
 *    the caller.  The library never allocates or frees device memory inside
 *    a call; scratch memory comes in through `workspace`.
 *  - Arrays are row-major, mixture-major: element (m, i) of an n x nc array
 *    is at m*nc + i; k_ij of a shared set is at i*nc + j.
 *  - Calls enqueue work on `stream` and return; results are valid once the
 *    stream has been synchronised.  The PLAIN form also synchronises the
 *    stream inside the call (it reads the active count after every stage
 *    iteration).
 *  - Return value: 0 on success or a PTFLASH_E* code; nothing is printed and
 *    no exception crosses the ABI.  On a non-zero code no output is
 *    guaranteed to be written.
 */
#ifndef PTFLASH_H_
#define PTFLASH_H_

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- call-level return codes ---- */
#define PTFLASH_OK 0
#define PTFLASH_EINVAL 1          /* null pointer, n < 0, bad option value     */
#define PTFLASH_EUNSUPPORTED 2    /* nc outside the compiled range, or layout  */
#define PTFLASH_EWORKSPACE 3      /* workspace smaller than required          */
#define PTFLASH_EHIP 4            /* a HIP runtime call failed                */

/* ---- per-mixture status bits (status[m]) ---- */
#define PTFLASH_ST_INVALID        0x0001u /* z_i <= 0, non-finite T/P/z, bad props */
#define PTFLASH_ST_SHORTCUT       0x0002u /* unstable by the initial tpd test (case 3) */
#define PTFLASH_ST_SA_RAN         0x0004u /* stability analysis was run (cases 1, 2) */
#define PTFLASH_ST_SA_UNCONV      0x0008u /* a stability trial hit its iteration cap */
#define PTFLASH_ST_SPLIT_TR       0x0010u /* the split needed the trust region */
#define PTFLASH_ST_SPLIT_UNCONV   0x0020u /* the split hit its iteration cap */
#define PTFLASH_ST_SPLIT_TRIVIAL  0x0040u /* the split collapsed to x = y */
#define PTFLASH_ST_SPLIT_FAILED   0x0080u /* substitution left beta in (0,1) */
#define PTFLASH_ST_RR_NO_ROOT     0x0100u /* all K on one side of 1 in the split */
#define PTFLASH_ST_SWAPPED        0x0200u /* phases re-labelled so that Z_y > Z_x */
#define PTFLASH_ST_STEP_CAP       0x0400u /* stopped by the per-mixture step cap */
#define PTFLASH_ST_HINTED         0x0800u /* label set by the caller's hint */
#define PTFLASH_ST_SPLIT_RESTART  0x1000u /* the split restarted from the composition
                                             that proved the instability (substitution
                                             left the two-phase region, or the first
                                             descent ended at a degenerate split) */

/* ---- iteration counters (iters[m*PTFLASH_NITERS + k]) ---- */
#define PTFLASH_IT_PRE 0        /* initial phase-split substitutions (<= 3)  */
#define PTFLASH_IT_SS_V 1       /* stability trial V, substitutions (<= 9)  */
#define PTFLASH_IT_TR_V 2       /* stability trial V, trust-region steps    */
#define PTFLASH_IT_SS_L 3       /* stability trial L, substitutions         */
#define PTFLASH_IT_TR_L 4       /* stability trial L, trust-region steps    */
#define PTFLASH_IT_SS_SPLIT 5   /* phase-split substitutions (<= 9)         */
#define PTFLASH_IT_TR_SPLIT 6   /* phase-split trust-region steps           */
#define PTFLASH_IT_POLISH 7     /* Newton refinement steps                  */
#define PTFLASH_NITERS 8

/* ---- execution forms ---- */
#define PTFLASH_FORM_PERSISTENT 0 /* one launch per stage; waves refill finished
                                     lanes.  With grid, block and the lanes
                                     options all 0, a batch of n mixtures runs
                                     as FUSED when n <= 150000 (nc <= 8) or
                                     n * nc <= 400000 (nc > 8)            */
#define PTFLASH_FORM_PLAIN 1      /* one launch per stage iteration + compaction */
#define PTFLASH_FORM_FUSED 2      /* one launch; a lane pair carries one mixture
                                     through every stage, its two stability
                                     trials side by side (small batches)  */

/* Problem description.  Every mixture has the same nc (2 <= nc <= the value
 * of ptflash_max_nc()).  props_per_mixture = 0: Tc, Pc, omega hold nc values
 * and kij nc*nc values shared by all mixtures; 1: they hold n*nc and n*nc*nc
 * values, one component set per mixture.  kij must be symmetric with a zero
 * diagonal (mixtures whose set is not are flagged INVALID).  z rows need not
 * be normalised (each is divided by its sum).  T in K, P and Pc in the same
 * pressure unit. */
typedef struct {
    int64_t n;
    int32_t nc;
    int32_t props_per_mixture;
    const double *z;      /* n*nc   */
    const double *T;      /* n      */
    const double *P;      /* n      */
    const double *Tc;     /* nc or n*nc      */
    const double *Pc;     /* nc or n*nc      */
    const double *omega;  /* nc or n*nc      */
    const double *kij;    /* nc*nc or n*nc*nc */
    /* Optional per-mixture inputs (NULL: none).  They are where an external
     * initializer or classifier (the paper's neural networks, Sec. 4) or the
     * result of a previous time step enters the flash. */
    const double *lnk0;   /* n*nc: initial ln K in place of Wilson's (eq.
                             wilson), wherever the flash uses it: the first
                             substitutions, the two stability trials
                             W = K z and W = z / K, and the split of a
                             hinted-unstable mixture (Sec. 4: the
                             initializer serves stability analysis and split).
                             A row with a non-finite value is INVALID. */
    const int8_t *hint;   /* n: 0 = known stable (single phase, no analysis),
                             1 = known unstable (the split starts at once from
                             lnk0, else Wilson's K, without the triage and
                             the stability analysis); other values: none.
                             Hinted mixtures carry status HINTED and tm NaN. */
} ptflash_problem;

/* Options; ptflash_default_options() fills the paper's values. */
typedef struct {
    int32_t max_pre_ss;    /* 3: initial split substitutions (Sec. 2.2.3)       */
    int32_t max_ss;        /* 9: substitution cap, stability and split (2.2.1-2) */
    int32_t max_tr_sa;     /* 20: stability trust-region cap (Algorithm 2)      */
    int32_t max_tr_split;  /* 30: split trust-region cap                         */
    int32_t max_polish;    /* 4: Newton refinement steps after convergence       */
    int32_t dem_every;     /* 3: dominant-eigenvalue acceleration period, 0 off  */
    double tol_sa_ss;      /* 1e-6: max |d tm/d W| (Sec. 2.2.1)                 */
    double tol_sa_tr;      /* 1e-6: max |g| of the stability trust region (B.1) */
    double tol_split_ss;   /* 1e-8: max |K_new/K - 1| (Sec. 2.2.2)              */
    double tol_split_tr;   /* 1e-8: max |dG/dn^V| (Sec. 2.2.2, B.2)             */
    double tol_polish;     /* 1e-13: refinement stops when max |dn^V| is below  */
    double eps_tm;         /* 1e-10: a trial is unstable when tm < -eps_tm       */
    int32_t form;          /* PTFLASH_FORM_*                                     */
    int32_t keep_factor;   /* 1: write the Cholesky factor for the backward     */
    int32_t block;         /* threads per block (64, 128, 256), 0 = tuned       */
    int32_t grid;          /* persistent blocks, 0 = fill the device            */
    int32_t lanes_per_mixture; /* trust-region stages of the persistent form:
                              0 = the library's tuned choice for nc, 1 = one
                              mixture per lane, 16 or 32 = one group of that
                              many lanes per mixture (lane i holds component
                              i; needs 8 <= nc <= lanes).  Other values, or a
                              group too small for nc: PTFLASH_EINVAL.  The
                              plain form always runs one mixture per lane. */
    int32_t lanes_split;   /* the same choice for the split trust-region stage
                              alone: 0 = the tuned choice when
                              lanes_per_mixture is 0, else lanes_per_mixture */
    int32_t lanes_ss;      /* the same choice for the two substitution stages
                              (stability trials and split) of the persistent
                              form: 0 = the tuned choice, 1, 16 or 32 */
} ptflash_options;

/* Outputs (device pointers).  label, beta, x, y are required; the others may
 * be NULL.  Single-phase mixtures get label 0, beta = -1, x = y = z/sum(z).
 * Two-phase mixtures get label 1, beta in (0,1), x the liquid-like and y the
 * vapour-like phase (y has the larger compressibility factor). */
typedef struct {
    int8_t *label;        /* n       */
    double *beta;         /* n       */
    double *x;            /* n*nc    */
    double *y;            /* n*nc    */
    int16_t *iters;       /* n*PTFLASH_NITERS, nullable */
    uint16_t *status;     /* n, nullable                 */
    uint32_t *flops;      /* n, nullable: algorithmic flops spent per mixture */
    double *factor;       /* n*nc*(nc+1)/2, required when keep_factor: packed
                             lower Cholesky factor (row i, col j<=i at
                             i*(i+1)/2+j) of the Hessian of G with respect to
                             the vapour mole numbers at the solution; written
                             for two-phase mixtures only */
    double *tm;           /* n, nullable: the value that decided stability --
                             for a mixture found unstable by the initial
                             substitutions (status SHORTCUT), the most negative
                             of tpd(x), tpd(y) and Delta G (Sec. 2.2.3); else
                             the smaller final modified tangent plane distance
                             of the two trials (eq. tm, with tm(z) = 0).  The
                             mixture is unstable iff tm < -eps_tm.  NaN for
                             invalid input. */
} ptflash_result;

/* Fills the defaults listed in ptflash_options. */
void ptflash_default_options(ptflash_options *opt);

/* Largest nc the library was compiled for. */
int32_t ptflash_max_nc(void);

/* Bytes of device workspace ptflash_flash needs for this problem and
 * options (depends on n, nc and form only).  Returns 0 for a malformed
 * problem. */
size_t ptflash_workspace_bytes(const ptflash_problem *prob, const ptflash_options *opt);

/* The flash.  `workspace` must hold ptflash_workspace_bytes() bytes of
 * device memory, aligned to 256 bytes; its contents on entry do not matter. */
int ptflash_flash(const ptflash_problem *prob, const ptflash_options *opt,
                  ptflash_result *res, void *workspace, size_t ws_bytes,
                  hipStream_t stream);

/* Stability analysis alone: the initial substitutions and their triage
 * (Sec. 2.2.3), then Michelsen's two trials (Sec. 2.2.1, Algorithm 2) for the
 * mixtures the triage leaves undecided -- the same arithmetic as the first
 * stages of ptflash_flash, without the phase split.  Writes label (1 =
 * unstable: two or more phases; 0 = stable), and, when non-NULL, tm, iters
 * (slots 0-4), status and flops; beta, x, y and factor are not written and may
 * be NULL.  keep_factor must be 0.  The workspace is that of ptflash_flash
 * (ptflash_workspace_bytes).  A mixture's label here equals whether
 * ptflash_flash sends it to the phase split. */
int ptflash_stability(const ptflash_problem *prob, const ptflash_options *opt,
                      ptflash_result *res, void *workspace, size_t ws_bytes,
                      hipStream_t stream);

/* Adjoint of the flash by the implicit function theorem on the converged
 * equal-fugacity system r(n^V; p) = ln y + ln phi(y) - ln x - ln phi(x) = 0,
 * with parameters p = (z, T, P, k).  (The paper differentiates the
 * Rachford-Rice root this way, Sec. 4.2.2; here the whole split is.)  Given
 * upstream cotangents g_beta (n), g_x, g_y (n*nc) of a forward result `fwd`
 * computed with keep_factor = 1, writes the vector-Jacobian products g_z
 * (n*nc, with respect to the unnormalised z), g_T (n), g_P (n) and g_kij.
 * kij_reduce = 1 (shared k only): g_kij holds nc*nc values, the sum over
 * mixtures; 0: g_kij holds n*nc*nc per-mixture values.  The k gradient is
 * symmetric: entry (i,j) is the derivative for a symmetric perturbation of
 * k_ij = k_ji, split equally between (i,j) and (j,i).  Single-phase mixtures
 * give g_z = (g_x + g_y) projected through the normalisation, g_T = g_P = 0
 * and zero k gradient.  Mixtures whose forward status has INVALID,
 * SPLIT_UNCONV or STEP_CAP get NaN gradients (and contribute nothing to a
 * reduced k gradient).  The sum over mixtures is deterministic (fixed order).
 * `workspace` must hold ptflash_backward_workspace_bytes() bytes (256-byte
 * aligned). */
int ptflash_flash_backward(const ptflash_problem *prob, const ptflash_options *opt,
                           const ptflash_result *fwd, const double *g_beta,
                           const double *g_x, const double *g_y, double *g_z,
                           double *g_T, double *g_P, double *g_kij, int32_t kij_reduce,
                           void *workspace, size_t ws_bytes, hipStream_t stream);

/* Bytes of device workspace ptflash_flash_backward needs. */
size_t ptflash_backward_workspace_bytes(const ptflash_problem *prob, int32_t kij_reduce);

/* Diagnostic evaluation of the SRK phase model used inside the flash at
 * given compositions c (n*nc, normalised inside) and conditions T, P (n
 * each): ln phi (n*nc), the chosen compressibility factor Z (n) and, when
 * `phi` is not NULL, the matrix of unit-mole composition derivatives
 * Phi_ij = n d ln phi_i / d n_j (n*nc*nc, full).  Shared component set only.
 * (Appendix A, eqs. cubic_Z, halley, lnphi.) */
int ptflash_eval_phase(int64_t n, int32_t nc, const double *c, const double *T,
                       const double *P, const double *Tc, const double *Pc,
                       const double *omega, const double *kij, double *lnphi,
                       double *Z, double *phi, hipStream_t stream);

/* A batch of mixtures with different component counts, each with its own
 * component set (packed, mixture-major).  Mixture m has nc_of[m] components
 * (2 <= nc_of[m] <= ptflash_max_nc()); its rows start at off[m] in z, Tc,
 * Pc, omega and in the outputs x, y (off[m+1] - off[m] = nc_of[m]), and its
 * nc_of[m]^2 block of k_ij (row-major, symmetric, zero diagonal) starts at
 * koff[m].  T and P hold one value per mixture.  nc_of, off (n+1 values)
 * and koff (n values) are device arrays like the rest. */
typedef struct {
    int64_t n;
    const int32_t *nc_of;   /* n      */
    const int64_t *off;     /* n + 1  */
    const int64_t *koff;    /* n      */
    const double *z;        /* off[n] */
    const double *T;        /* n      */
    const double *P;        /* n      */
    const double *Tc;       /* off[n] */
    const double *Pc;       /* off[n] */
    const double *omega;    /* off[n] */
    const double *kij;      /* sum of nc_of[m]^2 */
    const double *lnk0;     /* NULL or off[n]: initial ln K, packed like z
                               (the meaning of ptflash_problem.lnk0) */
    const int8_t *hint;     /* NULL or n: the meaning of ptflash_problem.hint */
} ptflash_ragged_problem;

/* Bytes of device workspace ptflash_flash_ragged needs (depends on n and
 * the form only). */
size_t ptflash_ragged_workspace_bytes(const ptflash_ragged_problem *prob,
                                      const ptflash_options *opt);

/* The flash of a ragged batch (the method of ptflash_flash applied to every
 * mixture with its own nc and component set).  The mixtures are grouped by
 * nc on the device (counting sort into per-nc id lists), each group is
 * gathered into a contiguous uniform-nc batch in the workspace, flashed in
 * the selected form, and its outputs are scattered back: label, beta, iters,
 * status and flops per mixture, x and y at off[m].  res->factor must be
 * NULL (keep_factor is not supported here).  Mixtures with nc_of[m] outside
 * [2, ptflash_max_nc()] or a row count off[m+1] - off[m] != nc_of[m] are
 * reported INVALID (label 0, beta = -1, x = y = the raw z row).  The call
 * synchronises the stream once, to read the group sizes. */
int ptflash_flash_ragged(const ptflash_ragged_problem *prob, const ptflash_options *opt,
                         ptflash_result *res, void *workspace, size_t ws_bytes,
                         hipStream_t stream);

/* Largest workspace, in bytes, of ptflash_flash_noalloc: the size of the
 * library's own device scratch buffer (one per GPU). */
#define PTFLASH_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* ptflash_flash for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same flash, with the library's own static device scratch buffer of
 * PTFLASH_NOALLOC_SCRATCH_BYTES bytes as its workspace instead of a
 * caller's.  The caller still passes inputs and outputs.  No device memory
 * is allocated or freed by this call (the buffer exists once per GPU, for
 * the life of the process; its address is looked up on the first call on
 * each device).  Returns PTFLASH_EWORKSPACE, without launching anything,
 * when ptflash_workspace_bytes(prob, opt) exceeds the buffer (about 10^5
 * mixtures at nc = 8, 4.8 * 10^4 at nc = 20, persistent form).  Every call
 * on one GPU uses that GPU's one buffer: calls that overlap in time on one
 * GPU (different streams or host threads) race and must not be issued.
 * Arguments, outputs and other error codes as ptflash_flash. */
int ptflash_flash_noalloc(const ptflash_problem *prob, const ptflash_options *opt,
                          ptflash_result *res, hipStream_t stream);

/* Text for a return code (static storage). */
const char *ptflash_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* PTFLASH_H_ */
