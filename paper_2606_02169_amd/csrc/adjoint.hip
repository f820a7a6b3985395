// Adjoint of the matrix-free map y = H(theta) x with H(theta) = sum_p theta_p h_p.
//
// For an upstream gradient g (= dL/dRe y + i dL/dIm y), the input gradient is H^dagger g, and H is
// Hermitian when every group h_p is (the conditions h_- = conj(h_+) of Sec. IV.A and
// conj(J^{ab}) = J^{bar a bar b} of Eq. pairham), so grad_x = H g is the same target-driven gather
// (Sec. II) applied to g.  The coupling gradient Re <g|h_p x> equals Re <h_p g|x> for Hermitian h_p, and
// (h_p g)_F is the sum of the row-F contributions of the channels of group p, each of them already
// formed while gathering H g.  One pass over the rows therefore gives both:
//     grad_x[F]       = sum_c theta_{p_c} t_c(F)                       t_c(F) = w_c f_c(F) g[F - Delta_c]
//     grad_theta[p]  += Re conj(t_c(F)) x[F]       for every channel c of group p
// (diagonal terms are channels with Delta = 0).  Per-parameter sums are reduced over each wave with a
// fixed butterfly, accumulated per wave in LDS in row order, summed per block in a fixed order, and the
// block partials are summed by a second kernel in a fixed order, so the result does not depend on
// scheduling.
#include "mrmf_internal.h"

namespace mrmf {
namespace {

constexpr int kAdjBlock = 256;
constexpr int kAdjParamChunk = 32;  // parameters accumulated per pass (LDS: 32 x 4 doubles)
constexpr int kAdjMaxGrid = 2048;
constexpr int kAdjRows = 4;  // rows per thread per iteration (1 when their digits would not fit in LDS)

constexpr int kAdjMaxLdsTable = 4096;  // doubles of per-term factor tables staged in LDS (32 KB)

// floor(n / d) for n < 2^32 with magic = ceil(2^64 / d)
__device__ __forceinline__ uint32_t div_magic32(uint32_t n, uint64_t magic) {
    return static_cast<uint32_t>(__umul64hi(magic, static_cast<uint64_t>(n)));
}

// One pass for parameters [p0, p0 + kAdjParamChunk); the pass with p0 == 0 also writes grad_x.  Every
// lane of a wave walks the same row slots (lanes past D carry zeros), so the contributions
// Re conj(t) x_F of each run of consecutive terms with one parameter are summed per lane, then over the
// wave with a fixed butterfly, and added by lane 0 to the wave's accumulator in LDS: the per-parameter
// state is one double per wave instead of one per thread, which keeps the occupancy of the gather high.
// v moved across lanes by one DPP pattern (rows outside row_mask contribute 0), one 32-bit half at a time
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(static_cast<uint32_t>(u)), CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(static_cast<uint32_t>(u >> 32)), CTRL, ROW_MASK, 0xf,
                                               false);
    return __builtin_bit_cast(double, (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) |
                                          static_cast<uint64_t>(static_cast<uint32_t>(lo)));
}

// Sum over the 64 lanes of a wave with a fixed pattern of DPP moves (lane pairs 1 and 2 apart, the half
// and full row mirrors, then the row broadcasts of lanes 15 and 31); the total ends in lane 63.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_move<0xB1, 0xf>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_move<0x4E, 0xf>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_move<0x141, 0xf>(v);  // row_half_mirror
    v += dpp_move<0x140, 0xf>(v);  // row_mirror: every lane holds its row's sum
    v += dpp_move<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_move<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return v;                      // lane 63: the wave's sum
}

template <bool WIDE, bool LDS_TAB, int R>
__global__ __launch_bounds__(kAdjBlock) void k_adjoint(PlanArgs p, const AdjTerm* __restrict__ terms, int n_terms,
                                                       const double* __restrict__ ftab_g, int n_ftab,
                                                       const double* __restrict__ theta,
                                                       const double2* __restrict__ x,
                                                       const double2* __restrict__ g,
                                                       double2* __restrict__ gx, int p0,
                                                       double* __restrict__ partial) {
    constexpr int kWaves = kAdjBlock / 64;
    __shared__ double acc[kAdjParamChunk][kWaves];
    // dynamic LDS: [factor tables when LDS_TAB][digits: N x (R * kAdjBlock) bytes]
    extern __shared__ double ltab[];
    uint8_t* dig_base = reinterpret_cast<uint8_t*>(ltab + (LDS_TAB ? n_ftab : 0));
    auto dig = [&](int site, int slot) -> uint8_t& { return dig_base[site * (R * kAdjBlock) + slot]; };
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < kAdjParamChunk * kWaves; i += kAdjBlock) acc[i / kWaves][i % kWaves] = 0.0;
    const double* ftab = ftab_g;
    if (LDS_TAB) {
        for (int i = tid; i < n_ftab; i += kAdjBlock) ltab[i] = ftab_g[i];
        ftab = ltab;
    }
    __syncthreads();
    const bool write_gx = p0 == 0;
    const int64_t stride = int64_t(gridDim.x) * kAdjBlock * R;
    // each thread carries R rows (r * kAdjBlock apart) through every term
    for (int64_t base = int64_t(blockIdx.x) * kAdjBlock * R; base < p.D; base += stride) {
        int64_t F[R];
        bool act[R];
        double2 xf[R], gf[R];
        double hr[R], hi[R];
        for (int r = 0; r < R; ++r) {
            F[r] = base + r * kAdjBlock + tid;
            act[r] = F[r] < p.D;
            const int slot = r * kAdjBlock + tid;
            if (act[r]) {
                if (WIDE) {
                    int64_t f = F[r];
                    for (int i = p.N - 1; i >= 0; --i) {  // Eq. decode, least significant site first
                        const int64_t d = p.site[i].d;
                        const int64_t q = f / d;
                        dig(i, slot) = static_cast<uint8_t>(f - q * d);
                        f = q;
                    }
                } else {
                    uint32_t f = static_cast<uint32_t>(F[r]);
                    for (int i = p.N - 1; i >= 0; --i) {
                        const uint32_t q = div_magic32(f, p.site[i].magic);
                        dig(i, slot) = static_cast<uint8_t>(f - q * static_cast<uint32_t>(p.site[i].d));
                        f = q;
                    }
                }
            } else {
                for (int i = 0; i < p.N; ++i) dig(i, slot) = 0;
            }
            xf[r] = act[r] ? x[F[r]] : make_double2(0.0, 0.0);
            gf[r] = act[r] ? g[F[r]] : make_double2(0.0, 0.0);
            hr[r] = 0.0;
            hi[r] = 0.0;
        }
        // consecutive terms of one parameter are summed per lane first: one wave sum per run
        double run = 0.0;
        int run_q = -1;
        for (int k = 0; k < n_terms; ++k) {
            const AdjTerm T = terms[k];
            const int q = T.param - p0;
            const int qq = q >= 0 && q < kAdjParamChunk ? q : -1;
            if (qq != run_q) {
                if (run_q >= 0) {
                    const double v = wave_sum(run);
                    if (lane == 63) acc[run_q][wave] += v;
                }
                run = 0.0;
                run_q = qq;
            }
            const double th = theta[T.param];
            double fa[R];
            double2 gs[R];
            for (int r = 0; r < R; ++r) {  // factors (zero where a source digit is out of range), then gathers
                const int slot = r * kAdjBlock + tid;
                fa[r] = ftab[T.ta + dig(T.a, slot)];
                if (T.b >= 0) fa[r] *= ftab[T.tb + dig(T.b, slot)];
                if (T.diag)
                    gs[r] = gf[r];
                else
                    gs[r] = (act[r] && fa[r] != 0.0) ? g[F[r] - T.delta] : make_double2(0.0, 0.0);  // Eq. sourceoffset
            }
            for (int r = 0; r < R; ++r) {
                const double tr = fa[r] * (T.wr * gs[r].x - T.wi * gs[r].y);
                const double ti = fa[r] * (T.wr * gs[r].y + T.wi * gs[r].x);
                hr[r] += th * tr;
                hi[r] += th * ti;
                if (qq >= 0) run += tr * xf[r].x + ti * xf[r].y;
            }
        }
        if (run_q >= 0) {
            const double v = wave_sum(run);
            if (lane == 63) acc[run_q][wave] += v;
        }
        if (write_gx)
            for (int r = 0; r < R; ++r)
                if (act[r]) gx[F[r]] = make_double2(hr[r], hi[r]);
    }
    __syncthreads();
    const int np = p.n_params - p0 < kAdjParamChunk ? p.n_params - p0 : kAdjParamChunk;
    if (tid < np) {  // fixed order over the block's waves
        double s = 0.0;
        for (int w = 0; w < kWaves; ++w) s += acc[tid][w];
        partial[int64_t(blockIdx.x) * p.n_params + p0 + tid] = s;
    }
}

constexpr int kFinBlock = 256;

// grad_theta[q] = sum over blocks b of partial[b][q]: one block per parameter, each thread a fixed strided
// subset of the blocks, then a fixed-order tree over the threads.
__global__ __launch_bounds__(kFinBlock) void k_adjoint_finalize(int nb, int n_params, const double* __restrict__ partial,
                                                              double* __restrict__ out) {
    __shared__ double red[kFinBlock];
    const int q = blockIdx.x, t = threadIdx.x;
    double s = 0.0;
    for (int b = t; b < nb; b += kFinBlock) s += partial[int64_t(b) * n_params + q];
    red[t] = s;
    __syncthreads();
    for (int h = kFinBlock / 2; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    if (t == 0) out[q] = red[0];
}

int adjoint_grid(int64_t D) {
    const int64_t b = (D + kAdjBlock - 1) / kAdjBlock;
    return static_cast<int>(b < kAdjMaxGrid ? b : kAdjMaxGrid);
}

}  // namespace
}  // namespace mrmf

// Scratch of mrmf_adjoint_z_noalloc: the per-block partial sums of the coupling gradients (at most
// 2048 blocks x 64 parameters).  One copy per GPU, for the life of the process.  Host code never passes
// the array's name to a kernel (on the host it is a stand-in, not a device address): the device address
// comes from hipGetSymbolAddress, once per device, and is kept in g_noalloc_ptr.
static __device__ __align__(256) double scratch[MRMF_ADJOINT_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace mrmf {
namespace {

constexpr size_t kNoAllocScratchBytes = MRMF_ADJOINT_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mtx;
void* g_noalloc_ptr[kMaxDevices] = {};

// device address of this device's copy of `scratch` (resolved on the first call on the device)
mrmf_status noalloc_scratch(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MRMF_E_HIP;
    if (dev < 0 || dev >= kMaxDevices) return MRMF_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_noalloc_mtx);
    if (g_noalloc_ptr[dev] == nullptr) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) {
            (void)hipGetLastError();
            return MRMF_E_HIP;
        }
        g_noalloc_ptr[dev] = ptr;
    }
    *out = g_noalloc_ptr[dev];
    return MRMF_OK;
}

// Argument checks shared by both entry points (no HIP call).
mrmf_status adjoint_check(mrmf_plan plan, const void* d_ws, const double* d_theta, const void* d_x, const void* d_g,
                          void* d_grad_x, double* d_grad_theta) {
    if (!plan || !d_ws || !d_x || !d_g || !d_grad_x) return MRMF_E_INVALID_ARG;
    if (plan->n_params > 0 && (!d_theta || !d_grad_theta)) return MRMF_E_INVALID_ARG;
    if (!plan->hermitian) return MRMF_E_NOT_HERMITIAN;
    if (!aligned(d_ws, 256) || !aligned(d_x, 16) || !aligned(d_g, 16) || !aligned(d_grad_x, 16))
        return MRMF_E_INVALID_ARG;
    const size_t vb = size_t(plan->D) * 16;
    if (ranges_overlap(d_g, vb, d_grad_x, vb) || ranges_overlap(d_x, vb, d_grad_x, vb)) return MRMF_E_INVALID_ARG;
    return MRMF_OK;
}

size_t adjoint_scratch_need(const mrmf_plan_t* plan) {
    return size_t(adjoint_grid(plan->D)) * size_t(plan->n_params > 0 ? plan->n_params : 1) * sizeof(double);
}

// The adjoint pass with its partial sums in `partial` (checked by the caller).  allow_compile: build the
// plan's generated gradient kernel on first use; else run it only when it is already built, and the
// generic pass otherwise (no module is loaded, so nothing is allocated).
mrmf_status adjoint_run(mrmf_plan plan, const void* d_ws, const double* d_theta, const void* d_x, const void* d_g,
                        void* d_grad_x, double* d_grad_theta, double* partial, bool allow_compile, hipStream_t s) {
    // generated form: one pass of the kernel generated for the plan, then the fixed-order reduction
    if (plan->n_params > 0 && plan->cfg[MRMF_DTYPE_Z].mode != MRMF_KERNEL_GENERIC &&
        (allow_compile ? grad_prepare(plan) == MRMF_OK : grad_built(plan))) {
        int nb = 0;
        const mrmf_status st = grad_launch(plan, d_theta, d_x, d_g, d_grad_x, partial, adjoint_grid(plan->D), &nb, s);
        if (st != MRMF_OK) return st;
        hipLaunchKernelGGL(k_adjoint_finalize, dim3(plan->n_params), dim3(kFinBlock), 0, s, nb, plan->n_params,
                           partial, d_grad_theta);
        return launch_status();
    }
    const PlanArgs a = plan_args(plan, d_ws);
    const int grid = adjoint_grid(plan->D);
    const double* theta = plan->n_params > 0 ? d_theta : partial;  // never read when there are no params
    const int passes = plan->n_params > 0 ? (plan->n_params + kAdjParamChunk - 1) / kAdjParamChunk : 1;
    const bool wide = plan->D > int64_t(0xffffffffu);
    const int n_ftab = static_cast<int>(plan->ftab.size()), n_terms = static_cast<int>(plan->adj.size());
    const bool lds_tab = n_ftab <= kAdjMaxLdsTable;
    const size_t tab_bytes = lds_tab ? sizeof(double) * n_ftab : 0;
    // several rows per thread only when the grid stays full (small lattices need every wave they can get)
    const int rows = tab_bytes + size_t(plan->N) * kAdjRows * kAdjBlock <= 60000 &&
                             plan->D >= int64_t(kAdjMaxGrid) * kAdjBlock * kAdjRows
                         ? kAdjRows
                         : 1;
    using K = void (*)(PlanArgs, const AdjTerm*, int, const double*, int, const double*, const double2*,
                       const double2*, double2*, int, double*);
    const K kern = rows == kAdjRows
                       ? (wide ? (lds_tab ? k_adjoint<true, true, kAdjRows> : k_adjoint<true, false, kAdjRows>)
                               : (lds_tab ? k_adjoint<false, true, kAdjRows> : k_adjoint<false, false, kAdjRows>))
                       : (wide ? (lds_tab ? k_adjoint<true, true, 1> : k_adjoint<true, false, 1>)
                               : (lds_tab ? k_adjoint<false, true, 1> : k_adjoint<false, false, 1>));
    const unsigned char* wsb = static_cast<const unsigned char*>(d_ws);
    const AdjTerm* terms = reinterpret_cast<const AdjTerm*>(wsb + plan->off_adj);
    const double* ftab = reinterpret_cast<const double*>(wsb + plan->off_ftab);
    for (int k = 0; k < passes; ++k) {
        const size_t lds = tab_bytes + size_t(plan->N) * rows * kAdjBlock;
        hipLaunchKernelGGL(kern, dim3(grid), dim3(kAdjBlock), lds, s, a, terms, n_terms, ftab, n_ftab, theta,
                           static_cast<const double2*>(d_x), static_cast<const double2*>(d_g),
                           static_cast<double2*>(d_grad_x), k * kAdjParamChunk, partial);
        const mrmf_status st = launch_status();
        if (st != MRMF_OK) return st;
    }
    if (plan->n_params > 0) {
        hipLaunchKernelGGL(k_adjoint_finalize, dim3(plan->n_params), dim3(kFinBlock), 0, s, grid, plan->n_params,
                           partial, d_grad_theta);
        return launch_status();
    }
    return MRMF_OK;
}

}  // namespace
}  // namespace mrmf

extern "C" {

mrmf_status mrmf_adjoint_scratch_bytes(mrmf_plan plan, size_t* bytes) {
    if (!plan || !bytes) return MRMF_E_INVALID_ARG;
    *bytes = size_t(mrmf::adjoint_grid(plan->D)) * size_t(plan->n_params > 0 ? plan->n_params : 1) * sizeof(double);
    return MRMF_OK;
}

mrmf_status mrmf_adjoint_z(mrmf_plan plan, const void* d_ws, const double* d_theta, const void* d_x,
                           const void* d_g, void* d_grad_x, double* d_grad_theta, void* d_scratch,
                           size_t scratch_bytes, mrmf_stream stream) {
    using namespace mrmf;
    if (!d_scratch || !aligned(d_scratch, 8)) return MRMF_E_INVALID_ARG;
    const mrmf_status chk = adjoint_check(plan, d_ws, d_theta, d_x, d_g, d_grad_x, d_grad_theta);
    if (chk != MRMF_OK) return chk;
    if (scratch_bytes < adjoint_scratch_need(plan)) return MRMF_E_WORKSPACE;
    return adjoint_run(plan, d_ws, d_theta, d_x, d_g, d_grad_x, d_grad_theta, static_cast<double*>(d_scratch), true,
                       static_cast<hipStream_t>(stream));
}

mrmf_status mrmf_adjoint_z_noalloc(mrmf_plan plan, const void* d_ws, const double* d_theta, const void* d_x,
                                   const void* d_g, void* d_grad_x, double* d_grad_theta, mrmf_stream stream) {
    using namespace mrmf;
    const mrmf_status chk = adjoint_check(plan, d_ws, d_theta, d_x, d_g, d_grad_x, d_grad_theta);
    if (chk != MRMF_OK) return chk;
    if (adjoint_scratch_need(plan) > kNoAllocScratchBytes) return MRMF_E_WORKSPACE;
    void* ptr = nullptr;
    const mrmf_status st = noalloc_scratch(&ptr);
    if (st != MRMF_OK) return st;
    // every block writes all its partial sums before the finalize reads them: nothing to clear
    return adjoint_run(plan, d_ws, d_theta, d_x, d_g, d_grad_x, d_grad_theta, static_cast<double*>(ptr), false,
                       static_cast<hipStream_t>(stream));
}

}  // extern "C"
