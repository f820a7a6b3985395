// Internal declarations shared by the library's translation units (host plan, kernels, drivers).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mrmf.h"

namespace mrmf {

constexpr int kMaxSites = 64;

// complex element type of a real type
template <typename R>
struct Cx;
template <>
struct Cx<double> {
    using T = double2;
};
template <>
struct Cx<float> {
    using T = float2;
};
constexpr int kMaxDim = 256;  // largest local dimension d_i

// Off-diagonal channel (a term with at least one ladder operator).  The source digit of site a is
// n_a - qa (Eq. src_digit_two_site); the source index is F - delta (Eq. sourceoffset).
struct alignas(16) DevChan {
    int32_t a, b;      // sites, b = -1 for a one-site channel
    int32_t opa, opb;  // MRMF_OP_*
    int32_t qa, qb;    // digit shifts (+1 raise, -1 lower, 0 diagonal factor)
    int32_t param, term;
    int64_t delta, pad;
    double wr, wi;
};
static_assert(sizeof(DevChan) == 64, "DevChan layout");

// Diagonal term (only Z / Z2 operators).
struct alignas(16) DevDiag {
    int32_t a, b, opa, opb;
    int32_t param, term, pad0, pad1;
    double wr, wi;
};
static_assert(sizeof(DevDiag) == 48, "DevDiag layout");

// One term for the adjoint kernel: sites, offsets of its factor tables (value at the target digit, zero
// where the source digit is out of range) in the plan's factor-table array, parameter, offset, weight.
struct alignas(16) AdjTerm {
    int32_t a, b;    // b = -1: one-site term
    int32_t ta, tb;  // table offsets
    int32_t param, diag;
    int64_t delta;
    double wr, wi;
};
static_assert(sizeof(AdjTerm) == 48, "AdjTerm layout");

// Per-site data: local dimension, offset of the site's local tables, multiplier M_i and the
// reciprocal used for division by d_i of numerators below 2^32 (q = hi64(magic * n)).
struct alignas(16) DevSite {
    int32_t d, tab;
    int32_t kind, pad;
    int64_t M;
    uint64_t magic;
};
static_assert(sizeof(DevSite) == 32, "DevSite layout");

// Kernel-side view of an uploaded plan (pointers into the caller's workspace).
struct PlanArgs {
    const DevSite* site;
    const DevChan* chan;
    const DevDiag* diag;
    const double* val;  // val[tab + n]: S_z eigenvalue m = n - s (spin) or occupation n (boson)
    const double* up;   // up[tab + n] = <n|R|n-1> for n >= 1 (R = S_+ or a^dagger), up[tab] = 0
    const int32_t* lofs;  // general one-site operator i: its table <n|O|n - q> at up[lofs[i] + n]
    int64_t D;
    int32_t N, n_chan, n_diag, n_params;
};

// Tiling of the index space used by the tiled kernels: sites [k_in, N) form the inner block of
// T_in = prod d_i consecutive rows; the outer sites index tiles.
struct Tiling {
    int32_t k_in = 0;
    int32_t T_in = 1;
};

// Site split of the specialized kernel: uniform [0, k_u), unrolled [k_u, k_in) with P_U digit
// combinations, inner [k_in, N) with T_in rows.
struct Tile {
    int k_u = 0, k_in = 0;
    int64_t T_in = 1, P_U = 1;
    int n_top = 0;     // sites [0, n_top) are unrolled too (their copies lie M_s rows apart)
    int64_t P_C = 1;   // combinations of the contiguous unrolled sites [k_u, k_in); P_U = P_C * d_0 ... d_(n_top-1)
};

// Kernel selection and shape knobs of one element type (MRMF_KERNEL_*, MRMF_TUNE_*).
struct KernelCfg {
    int32_t mode = MRMF_KERNEL_AUTO;
    int32_t inner = 0;    // inner sites, 0 = library's choice
    int32_t unroll = -1;  // unrolled sites, -1 = library's choice
    int32_t sched = MRMF_SCHED_WINDOWS, bskip = 0, group = 0, blocks_per_cu = 0, variant = MRMF_VARIANT_MASKED;
    int32_t wide = 0;  // 1 = 64-bit addresses even when 32-bit buffer offsets would do
    int32_t cheb_fused = 1;  // time propagation: fused Chebyshev-step kernel (c128 configuration only)
    int32_t cheb_merge = 1;  // time propagation: steps of a fixed H taken as one series (c128 configuration)
    int32_t waves_per_eu = 0;  // register budget hint for the generated kernel (0: the compiler's choice)
    int32_t far_nt = 0;  // > 0: gathers with |Delta| >= 2^far_nt bytes are non-temporal loads
    int32_t far_dir = 0;  // which of those: 0 both directions, 1 sources behind (Delta > 0), 2 ahead (Delta < 0)
    int32_t grad_blocks_per_cu = 0;  // blocks per CU of the generated gradient kernel (0: the default, 2)
    int32_t outer_first = 0;  // the k most significant sites vary fastest in the super-tile sweep
    int32_t unroll_top = 0;   // k: sites 0..k-1 join the unrolled copies of every super-tile
};

// Slot of the c128 kernel with the Chebyshev-step epilogue in mrmf_plan_t::spec (after the dtypes).
constexpr int kSlotCheb = 2;

// Largest parameter count the generated coupling-gradient kernel keeps in registers (one accumulator each).
constexpr int kGradMaxParams = 48;

// A kernel generated and compiled for one plan and element type (see jit.cpp).
struct SpecKernel {
    bool tried = false;
    bool ok = false;
    int device = -1;
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
    int32_t k_in = 0, k_u = 0, T_in = 0, P_U = 1, block = 0, grid = 0;
    int64_t n_tiles = 0;
    std::string log;
};

}  // namespace mrmf

struct mrmf_plan_t {
    int32_t N = 0;
    std::vector<int32_t> kind, k, d;
    std::vector<int64_t> M;
    int64_t D = 1;
    int32_t n_params = 0;
    uint32_t flags = 0;
    bool hermitian = false;  // every parameter group h_p equals its adjoint
    std::vector<mrmf::DevChan> chans;
    std::vector<mrmf::DevDiag> diags;
    std::vector<int32_t> tab;
    std::vector<int32_t> lsite, lshift, lofs;  // general one-site operators: site, shift, table offset in up
    std::vector<double> val, up;
    std::vector<mrmf_term> terms;  // input copy
    // device image
    std::vector<unsigned char> image;
    size_t off_site = 0, off_chan = 0, off_diag = 0, off_val = 0, off_up = 0, off_lofs = 0;
    // adjoint term list (diagonal terms first, then channels, input order within each) and factor tables
    std::vector<mrmf::AdjTerm> adj;
    std::vector<double> ftab;
    size_t off_adj = 0, off_ftab = 0;
    size_t ws_bytes = 0;
    mrmf::Tiling tiling;
    // kernel selection (MRMF_KERNEL_*) and the specialized kernels per element type
    // kernel selection and shape, per element type (MRMF_DTYPE_Z, MRMF_DTYPE_C)
    mrmf::KernelCfg cfg[3];       // [kSlotCheb]: shape of the Chebyshev-step kernel once set explicitly
    bool cheb_shape_set = false;  // else that kernel takes the c128 configuration
    mrmf::SpecKernel spec[3];  // c128, c64, c128 with the Chebyshev-step epilogue
    mrmf::SpecKernel grad;     // coupling-gradient kernel of the adjoint (c128)
    std::mutex mtx;
    ~mrmf_plan_t();
};

// A digit-sum sector of a plan's basis (sector.hip).
struct mrmf_sector_t {
    int32_t N = 0, Q = 0;
    int64_t Dr = 0;
    int32_t n_params = 0;
    bool hermitian = false;
    std::vector<int32_t> d;
    std::vector<int64_t> M;
    std::vector<mrmf::DevChan> chans;  // digit-sum preserving channels
    std::vector<mrmf::DevDiag> diags;
    std::vector<unsigned char> image;  // device image: sites, channels, diagonal terms, tables, rank tables
    size_t off_site = 0, off_chan = 0, off_diag = 0, off_val = 0, off_up = 0, off_lofs = 0, off_rt = 0, off_rto = 0;
    int32_t n_rt = 0;
    int64_t rt_max = 0;  // largest rank-table entry (32-bit LDS tables when below 2^31)
    // packed digits of every sector state, filled on the device by mrmf_sector_upload after the image: row r's
    // word (lab_bytes = 4 or 8 bytes) at off_lab + r lab_bytes holds site k's digit in lab_w[k] bits, site
    // N - 1 in the lowest bits and site 0 in the highest (the words increase with r); lab_bytes = 0 when the
    // sector has none (digits over 64 bits, 2^28 states or more, or a generic-mode plan)
    std::vector<int32_t> lab_w;
    int32_t lab_bytes = 0;
    size_t off_lab = 0;
    size_t ws_bytes = 0;
    // host copies for the generated kernel: rank tables (site k at rto[k], entry (q, v) at q (d_k + 1) + v)
    // and the factor tables <n|O|n - q> of every term (diagonal terms, then channels; a then b, d entries
    // each, zero where the source digit is out of range)
    std::vector<int64_t> rt, rto;
    std::vector<double> tfac;
    int32_t mode = MRMF_KERNEL_AUTO;  // the plan's kernel selection when the sector was made
    int32_t blocks_per_cu = 0;        // blocks per CU of the generated kernel's grid (0: as many as fit)
    int32_t group = 0;                // gathers issued together by the generated kernel (0: default)
    int32_t sched = 0;                // MRMF_SCHED_* of the generated kernel's rows over the XCDs
    int32_t cheb_merge = 1;           // propagation: consecutive steps of a fixed H as one longer step
    int32_t cheb_fused = 1;           // propagation: the generated kernel with the Chebyshev-step epilogue
    mrmf::SpecKernel gen[3];          // generated sector kernels: c128, c64, c128 with the Chebyshev step
    std::mutex mtx;
    ~mrmf_sector_t();
};

namespace mrmf {

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Plan view over an uploaded workspace.
inline PlanArgs plan_args(const mrmf_plan_t* p, const void* d_ws) {
    const unsigned char* b = static_cast<const unsigned char*>(d_ws);
    PlanArgs a;
    a.site = reinterpret_cast<const DevSite*>(b + p->off_site);
    a.chan = reinterpret_cast<const DevChan*>(b + p->off_chan);
    a.diag = reinterpret_cast<const DevDiag*>(b + p->off_diag);
    a.val = reinterpret_cast<const double*>(b + p->off_val);
    a.up = reinterpret_cast<const double*>(b + p->off_up);
    a.lofs = reinterpret_cast<const int32_t*>(b + p->off_lofs);
    a.D = p->D;
    a.N = p->N;
    a.n_chan = static_cast<int32_t>(p->chans.size());
    a.n_diag = static_cast<int32_t>(p->diags.size());
    a.n_params = p->n_params;
    return a;
}

inline bool aligned(const void* ptr, size_t a) { return (reinterpret_cast<uintptr_t>(ptr) % a) == 0; }

inline bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
    uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + nb && y < x + na;
}

inline mrmf_status hip_status(hipError_t e) { return e == hipSuccess ? MRMF_OK : MRMF_E_HIP; }

// Launch-time error check (after hipLaunchKernelGGL).
inline mrmf_status launch_status() { return hip_status(hipGetLastError()); }

// Specialized kernels (jit.cpp).  spec_launch returns MRMF_E_UNSUPPORTED when the plan does not
// qualify or compilation failed (the caller then uses the generic kernel under MRMF_KERNEL_AUTO).
mrmf_status spec_prepare(mrmf_plan_t* p, int dtype);
mrmf_status spec_launch(mrmf_plan_t* p, int dtype, const void* theta, const void* x, void* y, hipStream_t s,
                        const int32_t* d_skip);

// Entry points shared between translation units.
mrmf_status matvec_z_impl(mrmf_plan_t* p, const void* d_ws, const double* theta,
                          const void* x, void* y, hipStream_t s, const int32_t* d_skip);
mrmf_status matvec_c_impl(mrmf_plan_t* p, const void* d_ws, const float* theta,
                          const void* x, void* y, hipStream_t s, const int32_t* d_skip);
// A map x -> y enqueued on a stream (device pointers; `stopped` non-null: skip when the device flag is set).
using MatvecOp = std::function<mrmf_status(const void* x, void* y, hipStream_t s, const int32_t* stopped)>;
// Lanczos (the recurrence of mrmf_lanczos) for any map of dimension D; mv_c may be empty for MRMF_PREC_Z.
mrmf_status lanczos_scratch_bytes(int64_t D, int32_t m, int32_t precision, size_t* bytes);
mrmf_status lanczos_run(int64_t D, const MatvecOp& mv_z, const MatvecOp& mv_c, int32_t precision, int32_t m,
                        int32_t reorth, const void* d_v0, void* d_V, double* d_alpha, double* d_beta,
                        double* d_result, void* d_u, void* d_scratch, size_t scratch_bytes, mrmf_stream stream);
// Time propagation (the Chebyshev series of mrmf_propagate_z) for any Hermitian map of dimension n: mv
// applies it with the couplings of the current step (theta null when there are none); step, when not null,
// is a fused Chebyshev step (p = ea H cur + eb cur + eg prev; prev = p; acc += (cr + i ci) p), used when
// fused_ready() returns true; merge: consecutive steps of a fixed map are taken as one longer step.
using ThetaMatvecOp = std::function<mrmf_status(const double* theta, const void* x, void* y, hipStream_t s)>;
using ChebStepOp = std::function<mrmf_status(const double* theta, const void* cur, void* prev, void* acc,
                                             double ea, double eb, double eg, double cr, double ci, hipStream_t s)>;
size_t propagate_scratch_bytes(int64_t n);
mrmf_status propagate_run(int64_t n, int32_t n_params, const ThetaMatvecOp& mv, const ChebStepOp* step,
                          const std::function<bool()>& fused_ready, bool merge, const double* d_theta,
                          int64_t theta_stride, double dt, int32_t n_steps, double e_min, double e_max, double tol,
                          const void* d_x0, void* d_x, void* d_scratch, size_t scratch_bytes, int32_t* h_n_terms,
                          hipStream_t s);
// Generated source of the specialized kernel (no device needed); "" when the plan does not qualify.
std::string spec_source(const mrmf_plan_t* p, int dtype, Tile* tl, bool epi = false);
// Fused Chebyshev step (time propagation) with the specialized c128 kernel:
// p = ea (H x) + eb x + eg prev;  prev = p;  acc += (ecr + i eci) p.  MRMF_E_UNSUPPORTED when the plan
// has no specialized kernel.
mrmf_status spec_launch_cheb(mrmf_plan_t* p, const double* theta, const void* x, void* prev, void* acc, double ea,
                             double eb, double eg, double ecr, double eci, hipStream_t s);
// <n|O|n - q> of site's operator op at target digit n; 0 where the source digit is out of range
double local_factor_host(const mrmf_plan_t* p, int site, int op, int n);
// Adjoint kernel generated for the plan (jit.cpp): source ("" when the plan does not qualify), compilation,
// and a launch of at most max_grid blocks of 256 threads writing gx = H g and partial[block][param]
// (*grid: the blocks launched).  MRMF_E_UNSUPPORTED when the plan does not qualify.
std::string grad_source(const mrmf_plan_t* p);
// Sector kernel generated for one sector and element type (jit.cpp): "" when the sector does not qualify
// (no packed digits, tables over their LDS budget, or a vector of 2^31 bytes or more); launch returns
// MRMF_E_UNSUPPORTED then.  lab: the packed digits in the uploaded workspace.
std::string sector_source(const mrmf_sector_t* S, int dtype, bool epi = false);
// slot: MRMF_DTYPE_Z, MRMF_DTYPE_C, or kSectorSlotCheb (c128 with the Chebyshev-step epilogue:
// prev = ea (P H P^T x) + eb x + eg prev; acc += (ecr + i eci) prev, row by row)
constexpr int kSectorSlotCheb = 2;
mrmf_status sector_gen_prepare(mrmf_sector_t* S, int slot);
mrmf_status sector_gen_launch_cheb(mrmf_sector_t* S, const void* lab, const double* theta, const void* x, void* prev,
                                   void* acc, double ea, double eb, double eg, double ecr, double eci, hipStream_t s);
mrmf_status sector_gen_launch(mrmf_sector_t* S, int dtype, const void* lab, const void* theta, const void* x, void* y,
                              hipStream_t s, const int32_t* d_skip);
mrmf_status grad_prepare(mrmf_plan_t* p);
// true when the plan's generated gradient kernel is already built for the current device (compiles nothing)
bool grad_built(mrmf_plan_t* p);
mrmf_status grad_launch(mrmf_plan_t* p, const double* theta, const void* x, const void* g, void* gx, double* partial,
                        int max_grid, int* grid, hipStream_t s);

}  // namespace mrmf
