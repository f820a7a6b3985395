/*
 * mrmf — mixed-radix matrix-free spin/boson Hamiltonians on MI355X (gfx950).
 *
 * C ABI of the HIP library libmrmf.so.  The library applies y = H x for a lattice Hamiltonian given
 * as a list of local dimensions and a list of one- and two-site operator terms, without storing H
 * ("Spin Hamiltonian as Matrix-Free Linear Map", Sec. II target-driven form, Sec. III mixed-radix
 * indexing, Sec. IV one- and two-site rules, App. A pseudocode, App. B (S_z)^2 channel, App. C
 * truncated boson digits), drives it with a device-resident Lanczos eigensolver, applies its adjoint
 * for gradients, and runs many lattices in one persistent launch.
 *
 * Conventions common to every entry point
 * ---------------------------------------
 *  - Site 0 is the most significant digit: M_k = prod_{l>k} d_l, index = sum_k n_k M_k (Sec. III,
 *    Eq. encode), i.e. C-order flattening of a tensor of shape (d_0, .., d_{N-1}).
 *  - Local digit n = m + s for a spin (n = 0 is m = -s), n = occupation for a boson (App. C).
 *  - Complex vectors are interleaved (re, im): c128 = 2 x double, c64 = 2 x float.
 *  - Every pointer named d_* is DEVICE memory owned by the caller; the library never allocates device
 *    memory.  Host arrays are read during the call only.
 *  - Every call that takes a stream enqueues its work on that stream (a hipStream_t, passed as
 *    void*; NULL is the null stream) and returns without synchronising.  Argument errors are
 *    reported synchronously, before anything is enqueued; launch failures map to MRMF_E_HIP.
 *  - No C++ exception crosses this interface.
 */
#ifndef MRMF_H
#define MRMF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mrmf_status;
#define MRMF_OK 0
#define MRMF_E_INVALID_ARG (-1)   /* bad pointer, size, site index, operator, aliasing          */
#define MRMF_E_OVERFLOW (-2)      /* D = prod d_i >= 2^62 (single-word index bound, Sec. VI)      */
#define MRMF_E_NOT_HERMITIAN (-3) /* some parameter group h_p differs from its adjoint (IV.A, IV.B) */
#define MRMF_E_HIP (-4)           /* a HIP runtime call or kernel launch failed                  */
#define MRMF_E_UNSUPPORTED (-5)   /* valid request outside what the library implements           */
#define MRMF_E_WORKSPACE (-6)     /* workspace / scratch smaller than the size query returned     */

typedef void* mrmf_stream; /* hipStream_t */
typedef struct mrmf_plan_t* mrmf_plan;
typedef struct mrmf_batch_t* mrmf_batch;

/* Site kinds.  SPIN: k = 2s, local dimension d = k + 1 (Sec. I, Eq. 1).
 * BOSON: k = n_max, digits 0..n_max, d = k + 1 (App. C). */
#define MRMF_SPIN 0
#define MRMF_BOSON 1
typedef struct {
    int32_t kind;
    int32_t k;
} mrmf_site;

/* Local operators.  Z: S_z (spin) or a^dag a (boson); Z2: its square (App. B diagonal channel, one-site
 * only); RAISE: S_+ or a^dag (digit shift +1); LOWER: S_- or a (digit shift -1) (Sec. IV.A, App. C);
 * RAISE2 / LOWER2: (S_+)^2 / (S_-)^2, or a^dag^2 / a^2 (digit shift +2 / -2, one-site only: the q = +-2
 * local monomials of App. B, e.g. the E (S_x^2 - S_y^2) = (E/2)(S_+^2 + S_-^2) zero-field-splitting term),
 * coefficient the product of the two one-step ladder elements. */
#define MRMF_OP_Z 0
#define MRMF_OP_Z2 1
#define MRMF_OP_RAISE 2
#define MRMF_OP_LOWER 3
#define MRMF_OP_RAISE2 4
#define MRMF_OP_LOWER2 5
/* General one-site operators (App. B: any local monomial (S_+)^p (S_z)^r (S_-)^l, quadrupolar factors,
 * truncated local sets): MRMF_OP_LOCAL(i) names entry i of the local-operator list given to
 * mrmf_plan_create_ex.  Such an operator lives on one band: <n|O|n'> is nonzero only for n - n' = shift,
 * and values[n] = <n|O|n - shift> for the target digit n (entries whose source n - shift is outside
 * 0..d-1 are ignored).  It may appear in one-site terms and on either side of two-site terms (the general
 * alpha-beta channels), always on its own site. */
#define MRMF_OP_LOCAL_BASE 16
#define MRMF_OP_LOCAL(i) (MRMF_OP_LOCAL_BASE + (i))
typedef struct {
    int32_t site;          /* the site it acts on (its d gives the table length) */
    int32_t shift;         /* q in (-d, d) */
    const double* values;  /* host, d entries, read during mrmf_plan_create_ex only */
} mrmf_local_op;

/* One term of  H(theta) = sum_t theta[param_t] * (w_re + i w_im) * O_{op_a}^{(site_a)} O_{op_b}^{(site_b)}.
 * site_b = -1 makes it a one-site term (op_b ignored; op_a any MRMF_OP_*).  A two-site term needs
 * site_a != site_b and op_a, op_b in {Z, RAISE, LOWER}: the pair channels J^{alpha beta} of Eq. (pairham).  theta is real and
 * supplied per call in device memory, so couplings can change between calls without a new plan. */
typedef struct {
    int32_t site_a, op_a, site_b, op_b;
    int32_t param, reserved;
    double w_re, w_im;
} mrmf_term;

/* plan flags */
#define MRMF_REQUIRE_HERMITIAN 1u /* reject unless every group h_p = sum_{param_t = p} w_t O_t is Hermitian */

/* precision forms for mrmf_lanczos */
#define MRMF_PREC_Z 0       /* c128 matvec, FP64 everything                                   */
#define MRMF_PREC_C_IN_Z 1  /* c64 matvec on a c64 copy of v_j; FP64 dots, reorth, T solve     */

/* reorthogonalisation policies for mrmf_lanczos */
#define MRMF_REORTH_CGS2 0  /* full: classical Gram-Schmidt against all of V, applied twice       */
#define MRMF_REORTH_NONE 1  /* plain three-term recurrence                                       */
#define MRMF_REORTH_CGS2_COND 2 /* full: classical Gram-Schmidt, the second pass only when the first
                                   one shrank ||w|| by more than 1/sqrt(2) (Daniel, Gragg, Kaufman and
                                   Stewart's criterion; the decision is taken on the device) */
#define MRMF_REORTH_PARTIAL 3   /* partial (Simon 1984): the loss of orthogonality is estimated from
                                   alpha and beta, and one Gram-Schmidt pass against all of V runs only
                                   at the steps where an estimate passes sqrt(eps) and the step after */

/* ---------------------------------------------------------------------------------------------- */
/* Status text ("ok", "invalid argument", ...).  Static storage; never NULL. */
const char* mrmf_status_string(mrmf_status s);
/* Library version, major*10000 + minor*100 + patch. */
int32_t mrmf_version(void);

/* Build a plan (host only, no HIP call): validates sites and terms, computes d_i, the multipliers M_i
 * and D (Sec. III) with an overflow check (Sec. VI, index-range remark), folds the diagonal terms, and
 * lists the off-diagonal terms with their integer source offsets (Eq. sourceoffset) and closed-form
 * ladder tables (App. A Lambda).  n_sites in [1, 64]; every d_i in [2, 256]; params in [0, n_params).
 * flags: MRMF_REQUIRE_HERMITIAN.  On success *out owns host memory until mrmf_plan_destroy. */
mrmf_status mrmf_plan_create(int32_t n_sites, const mrmf_site* sites, int32_t n_terms,
                             const mrmf_term* terms, int32_t n_params, uint32_t flags, mrmf_plan* out);
/* The same with a list of general one-site operators (MRMF_OP_LOCAL(i), i < n_local <= 4096).  A term
 * may combine them with the built-in operators; Hermiticity (MRMF_REQUIRE_HERMITIAN) is then checked
 * numerically, band by band, against the adjoint of every group (relative tolerance 1e-12). */
mrmf_status mrmf_plan_create_ex(int32_t n_sites, const mrmf_site* sites, int32_t n_terms,
                                const mrmf_term* terms, int32_t n_params, uint32_t flags, int32_t n_local,
                                const mrmf_local_op* local, mrmf_plan* out);
void mrmf_plan_destroy(mrmf_plan plan);

/* Host *D = prod_i d_i, the dimension of the product basis (Sec. I, the first displayed equation; also
 * M_0 d_0 with the multipliers of Sec. III).  MRMF_E_INVALID_ARG for a null argument; no HIP call. */
mrmf_status mrmf_plan_dim(mrmf_plan plan, int64_t* D);
/* Number of off-diagonal terms (those with a RAISE or LOWER operator): the "channels". */
mrmf_status mrmf_plan_n_offdiag(mrmf_plan plan, int32_t* n);
/* For channel c (c = 0..n_offdiag-1, in input order): host out[c] = index of its input term. */
mrmf_status mrmf_plan_offdiag_terms(mrmf_plan plan, int32_t* out);
/* For channel c: host out[c] = Delta_c with source index I = F - Delta_c (Eq. sourceoffset:
 * Delta = delta(alpha) M_i + delta(beta) M_j). */
mrmf_status mrmf_plan_offsets(mrmf_plan plan, int64_t* out);

/* Device workspace the plan's tables need (bytes, 256-aligned).  The caller allocates it and fills it
 * once with mrmf_plan_upload (an async host-to-device copy on the stream); it is read-only afterwards
 * and may be shared by concurrent calls. */
mrmf_status mrmf_plan_workspace_bytes(mrmf_plan plan, size_t* bytes);
mrmf_status mrmf_plan_upload(mrmf_plan plan, void* d_ws, size_t ws_bytes, mrmf_stream stream);

/* Kernel selection for mrmf_matvec_z / mrmf_matvec_c (and everything that calls them).
 *   MRMF_KERNEL_GENERIC     : one data-driven kernel for every plan (tables read at run time).
 *   MRMF_KERNEL_SPECIALIZED : a kernel generated for this plan's structure (sites, channels, offsets and
 *                             ladder tables as compile-time constants; couplings theta still read per
 *                             call), compiled with hiprtc for the current device on first use.  Each
 *                             thread owns one row of the block of the low `inner_sites` sites and
 *                             handles every digit combination of the next `unrolled_sites` sites.
 *   MRMF_KERNEL_AUTO        : specialized when the plan qualifies (all buffer offsets, about
 *                             2 * D * element size, below 2^31 bytes), else generic.
 * inner_sites = 0 and unrolled_sites = -1 let the library choose.  Not thread-safe against concurrent
 * calls on the same plan. */
#define MRMF_KERNEL_AUTO 0
#define MRMF_KERNEL_GENERIC 1
#define MRMF_KERNEL_SPECIALIZED 2
/* element types of the plain matvec */
#define MRMF_DTYPE_Z 0 /* c128 */
#define MRMF_DTYPE_C 1 /* c64  */
mrmf_status mrmf_plan_set_kernel(mrmf_plan plan, int32_t kind, int32_t inner_sites, int32_t unrolled_sites);
/* Tuning knobs of the specialized kernel (each change makes the next call regenerate it):
 *   MRMF_TUNE_SCHEDULE      : MRMF_SCHED_WINDOWS  - the grid sweeps windows of consecutive super-tiles,
 *                                                   each XCD taking one eighth of every window;
 *                             MRMF_SCHED_XCD_CHUNK - each XCD sweeps its own contiguous eighth of the
 *                                                   super-tiles with its blocks side by side;
 *                             MRMF_SCHED_BLOCK_RUN - each block sweeps its own contiguous run of
 *                                                   super-tiles (runs of one XCD adjacent).
 *                             A sector made from the plan afterwards schedules its generated kernel's
 *                             groups of 256 rows the same way.
 *   MRMF_TUNE_BRANCH_SKIP   : 1 = a channel whose tile-uniform source digits are inadmissible is skipped
 *                             by a scalar branch; 0 = its loads are issued and masked.
 *   MRMF_TUNE_LOAD_GROUP    : channels whose gathers are issued ahead of their accumulation (0 = default);
 *                             a sector made from the plan afterwards uses it in its generated kernel.
 *   MRMF_TUNE_BLOCKS_PER_CU : cap on resident blocks per compute unit (0 = as many as fit); a sector
 *                             made from the plan afterwards sizes its generated kernel's grid with it.
 *   MRMF_TUNE_VARIANT       : MRMF_VARIANT_MASKED - every channel that reads outside the super-tile is
 *                                                   issued, masked when inadmissible;
 *                             MRMF_VARIANT_LIST   - those channels are compacted per super-tile into a
 *                                                   list of admissible ones that every thread walks
 *                                                   (MRMF_TUNE_LOAD_GROUP = gathers per chunk).
 *   MRMF_TUNE_ADDRESSING    : 0 = 32-bit buffer offsets while a vector (plus its gather reach) fits in
 *                             2 GiB, 64-bit global addresses beyond that (default); 1 = 64-bit addresses
 *                             always.  Either way every channel offset |Delta| plus a super-tile must stay
 *                             below 2^31 bytes, else the plan keeps the generic kernel.
 *   MRMF_TUNE_CHEB_FUSED    : 1 = mrmf_propagate_z runs each Chebyshev term as one launch of the
 *                             specialized kernel with the Chebyshev-step epilogue (default); 0 = a matvec
 *                             and a separate vector update per term.
 *   MRMF_TUNE_CHEB_MERGE    : 1 = mrmf_propagate_z takes consecutive steps of a fixed H (theta_stride 0)
 *                             as one step of their summed length, exp(-i H dt)^q = exp(-i H q dt), q as
 *                             large as keeps a series within 2048 terms (default); 0 = one series per
 *                             step.
 *   MRMF_TUNE_WAVES_PER_EU  : 0 = the compiler's register allocation (default); 1..8 = ask for at least
 *                             that many resident waves per SIMD (a register budget; may spill).
 *   MRMF_TUNE_FAR_LOADS     : 0 = every gather with the default cache policy (default); k in 10..40 = a
 *                             channel whose offset |Delta| spans at least 2^k bytes is loaded
 *                             non-temporal (the list form walks such channels first, from a list of their
 *                             own).  Results are unchanged.
 *   MRMF_TUNE_FAR_DIR       : which channels MRMF_TUNE_FAR_LOADS takes: 0 = both directions (default),
 *                             1 = sources behind the row (Delta > 0), 2 = sources ahead (Delta < 0).
 *   MRMF_TUNE_GRAD_BLOCKS_PER_CU : blocks of 256 threads per compute unit of the generated
 *                             coupling-gradient kernel of mrmf_adjoint_z (0 = default 2; 1..8).
 *   MRMF_TUNE_OUTER_FIRST   : 0 = super-tiles swept in index order (default); k in 1..8 = the digit
 *                             combinations of the k most significant sites (those that are uniform in
 *                             the tiling) are swept back to back, so a channel that moves one of them
 *                             reads a super-tile that a neighbouring block of the same XCD loads at the
 *                             same time (a periodic bond from site 0 to an inner site).  Any order
 *                             covers every row once; results are unchanged.
 *   MRMF_TUNE_UNROLL_TOP    : k in 1..3 = sites 0..k-1 join the unrolled copies: a super-tile is then
 *                             d_0 ... d_(k-1) runs of rows M_s apart, staged together in LDS, so a term
 *                             among those sites and the unrolled/inner sites (the closing bond of a ring
 *                             in site order) reads its source from LDS instead of a gather.  Needs more
 *                             than k uniform sites and at most 16 copies in all (else the generic
 *                             kernel); 0 = off (default).  Results are unchanged. */
#define MRMF_TUNE_SCHEDULE 0
#define MRMF_TUNE_BRANCH_SKIP 1
#define MRMF_TUNE_LOAD_GROUP 2
#define MRMF_TUNE_BLOCKS_PER_CU 3
#define MRMF_TUNE_VARIANT 4
#define MRMF_TUNE_ADDRESSING 5
#define MRMF_TUNE_CHEB_FUSED 6
#define MRMF_TUNE_WAVES_PER_EU 7
#define MRMF_TUNE_FAR_LOADS 8
#define MRMF_TUNE_GRAD_BLOCKS_PER_CU 9
#define MRMF_TUNE_OUTER_FIRST 10
#define MRMF_TUNE_UNROLL_TOP 11
#define MRMF_TUNE_FAR_DIR 12
#define MRMF_TUNE_CHEB_MERGE 13
#define MRMF_VARIANT_MASKED 0
#define MRMF_VARIANT_LIST 1
#define MRMF_SCHED_WINDOWS 0
#define MRMF_SCHED_XCD_CHUNK 1
#define MRMF_SCHED_BLOCK_RUN 2
mrmf_status mrmf_plan_set_tuning(mrmf_plan plan, int32_t knob, int32_t value);
/* Shape of the specialized kernel for one element type only (e.g. from a tuning cache): form
 * (MRMF_VARIANT_*), inner sites, unrolled sites, load group, top sites unrolled (0..3, MRMF_TUNE_UNROLL_TOP);
 * the other tuning knobs keep their values.  Selection becomes MRMF_KERNEL_AUTO for that
 * element type (the generic kernel runs when the shape does not fit).  mrmf_plan_set_kernel and
 * mrmf_plan_set_tuning set both element types.  dtype = MRMF_SOURCE_CHEB sets the shape of the
 * Chebyshev-step kernel of mrmf_propagate_z, which otherwise follows the c128 shape. */
mrmf_status mrmf_plan_set_shape(mrmf_plan plan, int32_t dtype, int32_t variant, int32_t inner_sites,
                                int32_t unrolled_sites, int32_t load_group, int32_t unroll_top);
/* Autotuner for the plain matvec: times every candidate shape of the specialized kernel (inner block of
 * 32..1024 rows, 0..2 unrolled sites, masked and list forms, list chunk 4/8/12; where a term joins site 0
 * to the unrolled/inner sites, also with sites 0 and 0..1 unrolled (MRMF_TUNE_UNROLL_TOP) in the masked
 * form and the list form with chunk 4) on the given buffers with HIP events on the stream (synchronising it),
 * keeps the fastest in the plan for this element type only (selection MRMF_KERNEL_AUTO) and writes host
 * out[0..5] = (variant, inner sites, unrolled sites, load group, microseconds per call, top sites
 * unrolled 0..2); the other tuning knobs return to their defaults.  y is
 * overwritten; x must not overlap y.  dtype = MRMF_SOURCE_CHEB tunes the Chebyshev-step kernel of
 * mrmf_propagate_z instead (c128, double theta); then d_y must hold 2 D c128 elements (the step's
 * previous-term and accumulator vectors), all overwritten. */
mrmf_status mrmf_plan_autotune(mrmf_plan plan, int32_t dtype, const void* d_ws, const void* d_theta,
                               const void* d_x, void* d_y, mrmf_stream stream, int32_t* out);
/* Build (compile and load) the kernel mrmf_matvec_z (dtype Z) or mrmf_matvec_c (dtype C) will use, now
 * rather than on the first call (e.g. before stream capture).  Synchronous; host-side only.
 * dtype = MRMF_SOURCE_GRAD builds the generated coupling-gradient kernel of mrmf_adjoint_z and returns
 * MRMF_E_UNSUPPORTED when the plan does not qualify for it (the adjoint then runs its generic pass). */
mrmf_status mrmf_plan_prepare(mrmf_plan plan, int32_t dtype);
/* Host out[0..7] = (kernel kind used, inner sites, rows per block T_in, block threads, grid blocks,
 * super-tiles, unrolled sites, unrolled copies) for the given dtype, after mrmf_plan_prepare. */
mrmf_status mrmf_plan_kernel_info(mrmf_plan plan, int32_t dtype, int32_t* out);
/* Source text of the specialized kernel for this plan and dtype, for inspection.  Host only.  Copies at
 * most cap - 1 bytes plus a NUL into buf (cap = 0: nothing is copied) and stores the full length in
 * *len.  MRMF_E_UNSUPPORTED when the plan does not qualify for the specialized kernel. */
#define MRMF_SOURCE_CHEB 2 /* dtype value of mrmf_plan_kernel_source: the c128 kernel with the fused
                             Chebyshev-step epilogue that mrmf_propagate_z launches */
#define MRMF_SOURCE_GRAD 3 /* dtype value of mrmf_plan_kernel_source only: the generated coupling-gradient
                             kernel of mrmf_adjoint_z */
mrmf_status mrmf_plan_kernel_source(mrmf_plan plan, int32_t dtype, char* buf, size_t cap, size_t* len);

/* y = H(theta) x, plain FP64 form.  d_theta: double[n_params]; d_x, d_y: c128[D], 16-byte aligned,
 * must not overlap (the gather form reads x while writing y, Sec. II).  y is overwritten (App. A). */
mrmf_status mrmf_matvec_z(mrmf_plan plan, const void* d_ws, const double* d_theta, const void* d_x,
                          void* d_y, mrmf_stream stream);
/* The same map y = H(theta) x (target-driven gather of Sec. II: digits by Eq. decode, channels by Eqs.
 * src_digit_two_site / sourceoffset, ladder factors of Sec. IV.A, App. B, App. C) in FP32: d_theta
 * float[n_params]; d_x, d_y c64[D], 8-byte aligned, must not overlap; y is overwritten; tables (the FP64
 * ladder values rounded once) and accumulation in FP32.  Errors as mrmf_matvec_z: MRMF_E_INVALID_ARG for
 * null, misaligned or overlapping buffers, MRMF_E_HIP when a launch fails. */
mrmf_status mrmf_matvec_c(mrmf_plan plan, const void* d_ws, const float* d_theta, const void* d_x,
                          void* d_y, mrmf_stream stream);

/* Integer part of the map, for bit-exact checks: for rows F0..F0+count-1 and every channel c,
 * d_out[(F - F0) * n_offdiag + c] = source index I of Eq. (sourceoffset) if both source digits are
 * admissible, else -1.  d_out: int64, device. */
mrmf_status mrmf_debug_sources(mrmf_plan plan, const void* d_ws, int64_t F0, int64_t count,
                               int64_t* d_out, mrmf_stream stream);

/* Adjoint of y = H(theta) x for an upstream gradient g = dL/dRe y + i dL/dIm y:
 *   d_grad_x     = H^dagger g = H g  (c128[D]; needs a Hermitian plan, Sec. IV.A/IV.B conditions)
 *   d_grad_theta = Re <g | h_p x>, p = 0..n_params-1  (double[n_params], h_p = dH/dtheta_p)
 * Two forms, both with deterministic block sums and a second-stage reduction in a fixed order: unless the
 * kernel selection is MRMF_KERNEL_GENERIC, d_grad_x comes from the plan's matvec applied to g and the
 * couplings from a kernel generated for the plan (parameter sums in registers; plans with 1..48
 * parameters and vectors below 2^31 bytes); otherwise, or when the plan does not qualify, one generic
 * gather pass over g computes both.
 * d_scratch: device memory of at least mrmf_adjoint_scratch_bytes.  d_grad_x must not overlap d_g or d_x. */
mrmf_status mrmf_adjoint_scratch_bytes(mrmf_plan plan, size_t* bytes);
mrmf_status mrmf_adjoint_z(mrmf_plan plan, const void* d_ws, const double* d_theta, const void* d_x,
                           const void* d_g, void* d_grad_x, double* d_grad_theta, void* d_scratch,
                           size_t scratch_bytes, mrmf_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving or training
 * loops, harnesses that forbid hipMalloc): mrmf_adjoint_z with the same arguments, results and checks, but
 * its scratch (the per-block partial sums of the coupling gradients) lives in a static device array of
 * MRMF_ADJOINT_NOALLOC_SCRATCH_BYTES per GPU that the library holds until the process ends.  The call
 * allocates nothing and compiles nothing: it runs the plan's generated gradient kernel only when that is
 * already built (mrmf_plan_prepare with MRMF_SOURCE_GRAD, or an earlier mrmf_adjoint_z), else the generic
 * pass.  The first call on a device resolves the array's device address (hipGetSymbolAddress): make it
 * outside graph capture.  MRMF_E_WORKSPACE when mrmf_adjoint_scratch_bytes(plan) exceeds the array.  All
 * calls on one GPU share its array (every call writes the partial sums it reads, so nothing carries over):
 * calls that overlap in time on one GPU (other streams, or other host threads) race and must be ordered by
 * the caller. */
#define MRMF_ADJOINT_NOALLOC_SCRATCH_BYTES (1u << 20)
mrmf_status mrmf_adjoint_z_noalloc(mrmf_plan plan, const void* d_ws, const double* d_theta, const void* d_x,
                                   const void* d_g, void* d_grad_x, double* d_grad_theta, mrmf_stream stream);

/* FP64 helpers on c128 vectors of length n (deterministic two-stage reductions; scratch from
 * mrmf_reduce_scratch_bytes):  d_out[0..1] = <a|b> (re, im);  d_out[0] = ||a||_2. */
mrmf_status mrmf_reduce_scratch_bytes(int64_t n, size_t* bytes);
mrmf_status mrmf_dot_z(int64_t n, const void* d_a, const void* d_b, double* d_out, void* d_scratch,
                       size_t scratch_bytes, mrmf_stream stream);
mrmf_status mrmf_norm_z(int64_t n, const void* d_a, double* d_out, void* d_scratch,
                        size_t scratch_bytes, mrmf_stream stream);

/* Device-resident Lanczos driving the matvec (the Krylov use of x -> H x, Sec. I).
 * Step j: w = H v_j; alpha_j = Re<v_j|w>; w -= alpha_j v_j + beta_{j-1} v_{j-1};
 * (MRMF_REORTH_CGS2) twice c = V^H w, w -= V c; (MRMF_REORTH_CGS2_COND) once, and a second time only
 * if that pass left ||w||^2 below half its value before it; (MRMF_REORTH_PARTIAL) once, only where
 * Simon's recurrence for the inner products <v_i|v_k> estimates one of them above sqrt(eps) and at the
 * step after such a step (the basis stays semi-orthogonal: every |<v_i|v_k>| up to about sqrt(eps));
 * eps is the machine epsilon of the matvec (FP64's, FP32's for MRMF_PREC_C_IN_Z);
 * beta_j = ||w||;
 * stop when beta_j <= 1e-14 * ||T|| (Gershgorin estimate);
 * v_{j+1} = w / beta_j.  Then the lowest eigenpair (theta, s) of the k x k tridiagonal T (bisection
 * and inverse iteration on the GPU), the unit Ritz vector u = V s / ||V s||, and the explicit residual
 * ||H u - theta u|| with the FP64 matvec.
 *   reorth   : MRMF_REORTH_CGS2, MRMF_REORTH_CGS2_COND, MRMF_REORTH_PARTIAL or MRMF_REORTH_NONE
 *   precision: MRMF_PREC_Z, or MRMF_PREC_C_IN_Z (then d_theta_c float[n_params] is required and the
 *              matvec runs in c64 on a c64 copy of v_j; everything else stays FP64)
 *   d_v0     : c128[D] start vector (normalised internally; zero norm -> steps = 0, theta = NaN)
 *   d_V      : c128[(m + 1) * D] Lanczos basis, caller-owned; row j is v_j
 *   d_alpha, d_beta : double[m]
 *   d_result : double[4] = theta, residual estimate beta_{k-1}|s_{k-1}|, explicit residual, steps k
 *   d_u      : c128[D] Ritz vector u = V s / ||V s|| (written; ||V s|| is 1 to rounding with full
 *              reorthogonalisation, 1 + O(sqrt(eps)) with the semi-orthogonal basis of
 *              MRMF_REORTH_PARTIAL, and can differ more without reorthogonalisation)
 *   d_scratch: at least mrmf_lanczos_scratch_bytes(plan, m, precision)
 * Requires a plan whose parameter groups are Hermitian (MRMF_E_NOT_HERMITIAN otherwise, checked before
 * any launch): the recurrence keeps only Re<v_j|H v_j>, so its Ritz values mean nothing for other H.
 * All work is enqueued on the stream; the host never waits inside the call. */
mrmf_status mrmf_lanczos_scratch_bytes(mrmf_plan plan, int32_t m, int32_t precision, size_t* bytes);
/* Work counts of the Lanczos above (Sec. I's Krylov use of x -> H x), for diagnostics: device int32
 * d_out[0..1] = (second Gram-Schmidt passes taken under MRMF_REORTH_CGS2_COND, Gram-Schmidt passes taken
 * under MRMF_REORTH_PARTIAL) by the mrmf_lanczos or mrmf_sector_lanczos call that last used d_scratch
 * (the same 256-B aligned pointer; enqueue on that call's stream, before the scratch is reused).  d_out:
 * 4-B aligned.  MRMF_E_INVALID_ARG for null or misaligned pointers. */
mrmf_status mrmf_lanczos_counts(const void* d_scratch, int32_t* d_out, mrmf_stream stream);
mrmf_status mrmf_lanczos(mrmf_plan plan, const void* d_ws, const double* d_theta_z,
                         const float* d_theta_c, int32_t precision, int32_t m, int32_t reorth,
                         const void* d_v0,
                         void* d_V, double* d_alpha, double* d_beta, double* d_result, void* d_u,
                         void* d_scratch, size_t scratch_bytes, mrmf_stream stream);

/* Time propagation x = exp(-i H dt)^n_steps x0 through the matvec (exact flat-basis propagation under
 * rebuilt or driven couplings, Sec. VII): each step applies the Chebyshev expansion
 *     exp(-i H dt) = exp(-i b dt) sum_k (2 - delta_k0) (-i)^k J_k(a dt) T_k((H - b) / a),
 * a = (e_max - e_min) / 2, b = (e_max + e_min) / 2, cut where 2 sum of the remaining |J_k(a dt)| <= tol;
 * one matvec and one fused vector update per term.  The spectrum of every step's H must lie in
 * [e_min, e_max] (else the series diverges): mrmf_spectral_bounds (device) or mrmf_plan_norm_bound (host,
 * symmetric, looser) give safe bounds.
 *   d_theta      : double[n_params] for step 0; step s uses d_theta + s * theta_stride (0 = fixed H;
 *                  n_params = a piecewise-constant drive stored step by step)
 *   dt           : step length (negative runs backwards); n_steps >= 0
 *   tol          : truncation bound relative to ||x0||, in (0, 1)
 *   d_x0, d_x    : c128[D]; d_x may equal d_x0 (in place) but may not partly overlap it
 *   d_scratch    : mrmf_propagate_scratch_bytes (three vectors), 256-B aligned
 *   h_n_terms    : host int32 (may be NULL): Chebyshev terms taken over the whole call (the series'
 *                  terms summed over the steps as taken; see MRMF_TUNE_CHEB_MERGE), known when the call
 *                  returns
 * Requires a plan whose parameter groups are Hermitian (MRMF_E_NOT_HERMITIAN otherwise);
 * MRMF_E_UNSUPPORTED when a step would need more than 2^20 terms. */
mrmf_status mrmf_propagate_scratch_bytes(mrmf_plan plan, size_t* bytes);
mrmf_status mrmf_propagate_z(mrmf_plan plan, const void* d_ws, const double* d_theta, int64_t theta_stride,
                             double dt, int32_t n_steps, double e_min, double e_max, double tol,
                             const void* d_x0, void* d_x, void* d_scratch, size_t scratch_bytes,
                             int32_t* h_n_terms, mrmf_stream stream);

/* Host-only: upper bound on ||H(theta)||_2, sum over terms of |theta_p w_t| ||O_a|| ||O_b|| (triangle
 * inequality; a one-site factor's norm is its largest matrix element).  h_theta: host double[n_params]. */
mrmf_status mrmf_plan_norm_bound(mrmf_plan plan, const double* h_theta, double* bound);

/* Gershgorin bounds of the spectrum of H(theta): d_out[0] <= every eigenvalue <= d_out[1] (device
 * double[2]), the extreme ends over the rows F of H_FF -+ R_F, with R_F the sum over the row's admissible
 * channels of |theta_p w f| (at least the row's off-diagonal sum).  One pass over the rows (no vector
 * read); usually much tighter than mrmf_plan_norm_bound, hence fewer Chebyshev terms in
 * mrmf_propagate_z.  Needs a plan whose parameter groups are Hermitian (MRMF_E_NOT_HERMITIAN otherwise).
 *   d_scratch : mrmf_spectral_bounds_scratch_bytes, 8-B aligned. */
mrmf_status mrmf_spectral_bounds_scratch_bytes(mrmf_plan plan, size_t* bytes);
mrmf_status mrmf_spectral_bounds(mrmf_plan plan, const void* d_ws, const double* d_theta, double* d_out,
                                 void* d_scratch, size_t scratch_bytes, mrmf_stream stream);
/* The same ends over count coupling vectors at once (a piecewise-constant drive, a parameter sweep):
 * d_out[0] <= every eigenvalue of H(theta_s) <= d_out[1] for s = 0 .. count - 1, theta_s at
 * d_theta + s * theta_stride (doubles; stride 0 repeats one vector).  One pass over the rows: since H is
 * linear in the couplings (Sec. I: H is a sum of local terms, here each carrying one coupling), a row's
 * diagonal entry is sum_p theta_p A_p and its channel radius sum_p |theta_p| B_p, with A_p and B_p taken
 * once per row from per-term tables in LDS; each further vector costs 2 n_params multiply-adds per row.
 * The ends equal the extremes of count calls of mrmf_spectral_bounds up to the order of the sums.
 * MRMF_E_UNSUPPORTED for plans with more than 8 couplings, more than 256 terms or term tables of more
 * than 2048 entries (call mrmf_spectral_bounds per vector then); count >= 1, theta_stride >= 0.
 *   d_scratch : mrmf_spectral_bounds_scratch_bytes, 8-B aligned. */
mrmf_status mrmf_spectral_bounds_many(mrmf_plan plan, const void* d_ws, const double* d_theta, int64_t theta_stride,
                                      int32_t count, double* d_out, void* d_scratch, size_t scratch_bytes,
                                      mrmf_stream stream);

/* Host-only: the Bessel weights J_0(z) .. J_{K}(z) (z >= 0) used by mrmf_propagate_z, with K the smallest
 * index whose tail 2 sum_{k > K} |J_k(z)| is <= tol; *n_terms = K + 1 and h_out (may be NULL, else at
 * least cap doubles) receives them.  MRMF_E_UNSUPPORTED when more than cap terms would be needed. */
mrmf_status mrmf_cheb_bessel(double z, double tol, int32_t cap, double* h_out, int32_t* n_terms);

/* Restricted basis of a globally constrained sector (Sec. VI, case 2; App. D): the product states whose
 * local digits sum to digit_sum (a spin digit is n = m + s, so a fixed total magnetization M is
 * digit_sum = M + sum_i s_i; with bosons the digit sum is the excitation number).  Sector vectors are
 * packed in ascending full-basis order (site 0 most significant); the packed position of a state is its
 * combinatorial rank (the Lehmer-code-style lookup of Sec. VI.B), so source rows are found without a
 * table of labels or a search.
 * The sector matvec is y = P H P^T x: channels whose source leaves the sector (every one-site ladder
 * channel, and pair channels with q_a + q_b != 0) contribute nothing and are dropped at creation.
 * mrmf_sector_create copies what it needs from the plan (the plan may be destroyed afterwards);
 * MRMF_E_INVALID_ARG for digit_sum outside 0 .. sum_i (d_i - 1) or a maximal digit sum above 65535.
 * Workspace: caller-owned, 256-B aligned, mrmf_sector_workspace_bytes, filled by mrmf_sector_upload
 * (stream-ordered: a copy of the tables, then, unless the plan's kernel selection was MRMF_KERNEL_GENERIC,
 * a kernel that writes every state's local digits packed into one 4- or 8-byte word, the inverse of the
 * rank that the generated kernel reads instead of unranking its rows; none when the digits take more than
 * 64 bits or the sector has 2^28 states or more). */
typedef struct mrmf_sector_t* mrmf_sector;
mrmf_status mrmf_sector_create(mrmf_plan plan, int32_t digit_sum, mrmf_sector* out);
void mrmf_sector_destroy(mrmf_sector sector);
mrmf_status mrmf_sector_dim(mrmf_sector sector, int64_t* dim);
mrmf_status mrmf_sector_workspace_bytes(mrmf_sector sector, size_t* bytes);
mrmf_status mrmf_sector_upload(mrmf_sector sector, void* d_ws, size_t ws_bytes, mrmf_stream stream);
/* y = P H(theta) P^T x on packed sector vectors (c128 / c64, 16-B / 8-B aligned, not overlapping).
 * Unless the plan's kernel selection was MRMF_KERNEL_GENERIC when the sector was made, the first call
 * per element type and device generates and compiles a kernel for this sector (sites, channels, factor
 * tables and rank-change tables compiled in); sectors that do not qualify (no packed digits, rank-change
 * tables over 40 KB or coefficient tables over 32 KB, vectors of 2^31 bytes or more) and generic-mode
 * sectors run the generic kernel. */
mrmf_status mrmf_sector_matvec_z(mrmf_sector sector, const void* d_ws, const double* d_theta, const void* d_x,
                                 void* d_y, mrmf_stream stream);
mrmf_status mrmf_sector_matvec_c(mrmf_sector sector, const void* d_ws, const float* d_theta, const void* d_x,
                                 void* d_y, mrmf_stream stream);
/* Host *used = 1 when the matvec of this element type (MRMF_DTYPE_Z / MRMF_DTYPE_C) runs the generated
 * sector kernel (built now if it was not yet), 0 when it runs the generic one.  Synchronous. */
mrmf_status mrmf_sector_generated(mrmf_sector sector, int32_t dtype, int32_t* used);
/* Source text of the generated sector kernel, for inspection; buffer contract of mrmf_plan_kernel_source.
 * dtype MRMF_DTYPE_Z / MRMF_DTYPE_C, or MRMF_SOURCE_CHEB for the c128 kernel with the Chebyshev-step
 * epilogue that mrmf_sector_propagate_z runs.  MRMF_E_UNSUPPORTED when the sector does not qualify.  Host
 * only. */
mrmf_status mrmf_sector_kernel_source(mrmf_sector sector, int32_t dtype, char* buf, size_t cap, size_t* len);
/* d_out[i] = full-basis index of packed row r0 + i (int64, device); d_scratch: >= 8 N bytes of device
 * memory the call may overwrite. */
mrmf_status mrmf_sector_labels(mrmf_sector sector, const void* d_ws, int64_t r0, int64_t count, int64_t* d_out,
                               void* d_scratch, size_t scratch_bytes, mrmf_stream stream);
/* Membership test: d_out[i] = packed row of full-basis index d_F[i], or -1 when it is not a sector state
 * (including indices outside 0 .. D-1). */
mrmf_status mrmf_sector_lookup(mrmf_sector sector, const void* d_ws, const int64_t* d_F, int64_t count,
                               int64_t* d_out, mrmf_stream stream);
/* Lanczos in the sector: the arguments, results and the Hermiticity requirement of mrmf_lanczos, with
 * vectors of the sector's dimension. */
mrmf_status mrmf_sector_lanczos_scratch_bytes(mrmf_sector sector, int32_t m, int32_t precision, size_t* bytes);
mrmf_status mrmf_sector_lanczos(mrmf_sector sector, const void* d_ws, const double* d_theta_z,
                                const float* d_theta_c, int32_t precision, int32_t m, int32_t reorth,
                                const void* d_v0, void* d_V, double* d_alpha, double* d_beta, double* d_result,
                                void* d_u, void* d_scratch, size_t scratch_bytes, mrmf_stream stream);
/* Gershgorin bounds of the spectrum of P H(theta) P^T: d_out[0] <= every eigenvalue <= d_out[1] (device
 * double[2]), the extreme ends over the sector's rows r of H_rr -+ R_r, with R_r the sum of |theta_p w f|
 * over the row's off-diagonal channels whose source digits are in range (every such source lies in the
 * sector: the channels keep the digit sum).  One device pass over the sector's rows, digits by unranking,
 * no vector read; usually tighter than the plan's bounds (mrmf_spectral_bounds), which contain the
 * sector's spectrum as well.  MRMF_E_NOT_HERMITIAN unless the sector's groups are Hermitian.
 *   d_theta   : double[n_params] on the device.
 *   d_scratch : mrmf_sector_spectral_bounds_scratch_bytes, 8-B aligned; d_out 8-B aligned. */
mrmf_status mrmf_sector_spectral_bounds_scratch_bytes(mrmf_sector sector, size_t* bytes);
mrmf_status mrmf_sector_spectral_bounds(mrmf_sector sector, const void* d_ws, const double* d_theta, double* d_out,
                                        void* d_scratch, size_t scratch_bytes, mrmf_stream stream);
/* The sector's ends over count coupling vectors in one pass, as mrmf_spectral_bounds_many is for the plan
 * (same arguments, limits and MRMF_E_UNSUPPORTED); d_scratch: mrmf_sector_spectral_bounds_scratch_bytes. */
mrmf_status mrmf_sector_spectral_bounds_many(mrmf_sector sector, const void* d_ws, const double* d_theta,
                                             int64_t theta_stride, int32_t count, double* d_out, void* d_scratch,
                                             size_t scratch_bytes, mrmf_stream stream);
/* Time propagation inside the sector, x = exp(-i P H P^T dt)^n_steps x0 on packed vectors (the restricted
 * basis as the way to shrink the propagated state, Sec. VI and Sec. VIII): the arguments, the Chebyshev
 * series, the merging of fixed-H steps (as the plan's MRMF_TUNE_CHEB_MERGE was when the sector was made)
 * and the Hermiticity requirement of mrmf_propagate_z, with vectors of the sector's dimension.  Each term
 * is one launch of the sector's generated kernel with a Chebyshev-step epilogue (the row's phi_{k-2} and
 * accumulator read and written in the same pass, as the plan's MRMF_TUNE_CHEB_FUSED was when the sector
 * was made), or a sector matvec and a fused vector update for sectors on the generic kernel.  Since H keeps
 * the digit sum, P H P^T is H on the sector
 * and this equals the full-basis propagation of a vector supported on the sector.  Bounds: the sector's own
 * (mrmf_sector_spectral_bounds), or the plan's (mrmf_spectral_bounds, mrmf_plan_norm_bound), since the
 * spectrum of P H P^T lies inside that of H (Cauchy interlacing).  d_scratch: mrmf_sector_propagate_scratch_bytes (three sector vectors),
 * 256-B aligned. */
mrmf_status mrmf_sector_propagate_scratch_bytes(mrmf_sector sector, size_t* bytes);
mrmf_status mrmf_sector_propagate_z(mrmf_sector sector, const void* d_ws, const double* d_theta, int64_t theta_stride,
                                    double dt, int32_t n_steps, double e_min, double e_max, double tol,
                                    const void* d_x0, void* d_x, void* d_scratch, size_t scratch_bytes,
                                    int32_t* h_n_terms, mrmf_stream stream);

/* Batched form: n independent lattices (plans), each applied to a block of nvec c64 vectors stored
 * row-major as [D_b][nvec] (row F of lattice b holds its nvec amplitudes contiguously), all in one
 * persistent launch.  Lattice b's block starts at element offset off_b (host query; offsets are
 * multiples of 32 elements).  d_theta_all: float, the n_params of lattice 0, then lattice 1, ...
 * (host query mrmf_batch_theta_offsets; the array must hold at least the last offset's count of
 * floats).  nvec in {1, 2, 4, 8}; at most 2048 lattices, each of at most 32 sites, 128 terms and 128
 * couplings, with D_b * nvec < 2^30.
 * The batch copies what it needs from the plans at creation; the plans may be destroyed afterwards. */
mrmf_status mrmf_batch_create(int32_t n, const mrmf_plan* plans, int32_t nvec, mrmf_batch* out);
void mrmf_batch_destroy(mrmf_batch batch);
mrmf_status mrmf_batch_total_elems(mrmf_batch batch, int64_t* elems); /* sum over b of D_b * nvec, padded */
mrmf_status mrmf_batch_offsets(mrmf_batch batch, int64_t* out);       /* host int64[n] */
mrmf_status mrmf_batch_theta_offsets(mrmf_batch batch, int32_t* out); /* host int32[n + 1] */
mrmf_status mrmf_batch_workspace_bytes(mrmf_batch batch, size_t* bytes);
mrmf_status mrmf_batch_upload(mrmf_batch batch, void* d_ws, size_t ws_bytes, mrmf_stream stream);
/* Y_b = H_b X_b for every lattice b, one launch.  d_X, d_Y: 16-byte aligned (8-byte when nvec = 1), not
 * overlapping; d_ws 256-byte aligned. */
mrmf_status mrmf_batch_matvec_c(mrmf_batch batch, const void* d_ws, const float* d_theta_all,
                                const void* d_X, void* d_Y, mrmf_stream stream);
/* Capture the batched launch (and its work-list reset) into a hipGraph owned by the batch, for the
 * given pointers; mrmf_batch_graph_launch replays it on a stream.  Re-capturing replaces the graph. */
mrmf_status mrmf_batch_graph_capture(mrmf_batch batch, const void* d_ws, const float* d_theta_all,
                                     const void* d_X, void* d_Y, mrmf_stream stream);
mrmf_status mrmf_batch_graph_launch(mrmf_batch batch, mrmf_stream stream);
/* Autotuner: times each candidate launch shape (tile-row limit, threads per block, schedule) on the
 * given buffers with HIP events, keeps the fastest for this batch, and writes host out[0..2] = (tile-row
 * limit, block threads, candidate index); mrmf_batch_get_shape reports the schedule chosen.
 * Synchronises the stream. */
mrmf_status mrmf_batch_autotune(mrmf_batch batch, const void* d_ws, const float* d_theta_all,
                                const void* d_X, void* d_Y, mrmf_stream stream, int32_t* out);
/* Set a launch shape directly (e.g. from a tuning cache).  Each lattice's rows are cut into tiles spanned
 * by its low sites, of at most tile_rows_max rows, one of (64, 128, 256, 512) * 8 / nvec; a block holds
 * max(1, block / T) such tiles in LDS at a time.  block_threads: a multiple of 64, at most 512 and at
 * most 4096 / nvec. */
mrmf_status mrmf_batch_set_shape(mrmf_batch batch, int32_t tile_rows_max, int32_t block_threads);
/* Work schedule of the persistent grid over the work items (a block's tiles, numbered lattice by
 * lattice): MRMF_BATCH_SCHED_RUNS (default) - each block takes a contiguous run of items, the runs of
 * one XCD adjacent; MRMF_BATCH_SCHED_WINDOWS - the grid sweeps windows of consecutive items, each XCD
 * taking one eighth of every window, so that the items one XCD holds at a time are neighbours (their
 * cross-tile gathers meet in that XCD's L2); MRMF_BATCH_SCHED_XCD_CHUNK - each XCD sweeps its own
 * contiguous eighth of the items with its blocks side by side.  Results are identical. */
#define MRMF_BATCH_SCHED_RUNS 0
#define MRMF_BATCH_SCHED_WINDOWS 1
#define MRMF_BATCH_SCHED_XCD_CHUNK 2
mrmf_status mrmf_batch_set_schedule(mrmf_batch batch, int32_t sched);
/* Host out[0..3] = (tile-row limit, block threads, schedule, grid blocks) of the current launch shape. */
mrmf_status mrmf_batch_get_shape(mrmf_batch batch, int32_t* out);
/* Shared input (on = 1), for parameter sweeps and disorder averages (many couplings on one structure,
 * Sec. VII): every lattice reads its input rows from the one block [D][nvec] at the start of d_X (which
 * then needs only that block: D * nvec elements, padded to the next multiple of 32), and the work items
 * are taken tile by tile across the lattices, so that the items worked on together read the same input
 * rows and gather windows.  Outputs stay in their own blocks of d_Y; each Y_b equals what the batch
 * computes from a copy of the block in every X_b, bit for bit.  MRMF_E_UNSUPPORTED unless every lattice
 * has the same local dimensions (then the same tiles).  on = 0 restores separate inputs.  A captured graph
 * keeps the mode it was captured with. */
mrmf_status mrmf_batch_share_input(mrmf_batch batch, int32_t on);
/* Parameter sweep by linearity: H(theta) = sum_p theta_p h_p (each term carries one coupling, Sec. I), so
 * the products of one structure at K coupling vectors are Y_k = sum_p theta_kp G_p with G_p = h_p X.
 * Given the P group products G_p (c64, n entries each, G_p at d_G + p * g_stride elements; e.g. the output
 * of a batch of P copies of the plan with a shared input and unit coupling vectors), this writes
 * Y_k[i] = sum_p d_theta[k * P + p] G_p[i] to d_Y + k * y_stride for k < K (c64; d_theta: float[K][P] on
 * the device).  One pass, bound by the writes of the K outputs; results equal the direct products up to
 * the order of the FP32 sums.  1 <= P <= 16, K >= 1, strides >= n; 8-byte aligned, G and Y not
 * overlapping. */
mrmf_status mrmf_sweep_combine_c(const float* d_theta, int32_t K, int32_t P, int64_t n, const void* d_G,
                                 int64_t g_stride, void* d_Y, int64_t y_stride, mrmf_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* MRMF_H */
