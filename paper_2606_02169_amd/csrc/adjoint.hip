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
// (diagonal terms are channels with Delta = 0).  Per-parameter sums are kept per thread in LDS, summed
// per block in a fixed order, and the block partials are summed by a second kernel in a fixed order, so
// the result does not depend on scheduling.
#include "mrmf_internal.h"

namespace mrmf {
namespace {

constexpr int kAdjBlock = 128;
constexpr int kAdjParamChunk = 32;  // parameters accumulated per pass (LDS: 32 x 128 doubles)
constexpr int kAdjMaxGrid = 2048;

__device__ __forceinline__ double local_factor64(const PlanArgs& p, int op, int tab, int n) {
    switch (op) {
        case MRMF_OP_Z: return p.val[tab + n];
        case MRMF_OP_Z2: return p.val[tab + n] * p.val[tab + n];
        case MRMF_OP_RAISE: return p.up[tab + n];
        case MRMF_OP_LOWER: return p.up[tab + n + 1];
        case MRMF_OP_RAISE2: return p.up[tab + n] * p.up[tab + n - 1];
        case MRMF_OP_LOWER2: return p.up[tab + n + 1] * p.up[tab + n + 2];
        default: return p.up[p.lofs[op - MRMF_OP_LOCAL_BASE] + n];  // general one-site operator
    }
}

// floor(n / d) for n < 2^32 with magic = ceil(2^64 / d)
__device__ __forceinline__ uint32_t div_magic32(uint32_t n, uint64_t magic) {
    return static_cast<uint32_t>(__umul64hi(magic, static_cast<uint64_t>(n)));
}

// One pass for parameters [p0, p0 + kAdjParamChunk); the pass with p0 == 0 also writes grad_x.
template <bool WIDE>
__global__ __launch_bounds__(kAdjBlock) void k_adjoint(PlanArgs p, const double* __restrict__ theta,
                                                       const double2* __restrict__ x,
                                                       const double2* __restrict__ g,
                                                       double2* __restrict__ gx, int p0,
                                                       double* __restrict__ partial) {
    __shared__ uint8_t dig[kMaxSites][kAdjBlock];
    __shared__ double acc[kAdjParamChunk][kAdjBlock];
    const int tid = threadIdx.x;
    for (int q = 0; q < kAdjParamChunk; ++q) acc[q][tid] = 0.0;
    const bool write_gx = p0 == 0;
    const int64_t stride = int64_t(gridDim.x) * kAdjBlock;
    for (int64_t F = int64_t(blockIdx.x) * kAdjBlock + tid; F < p.D; F += stride) {
        if (WIDE) {
            int64_t f = F;
            for (int i = p.N - 1; i >= 0; --i) {  // Eq. decode, least significant site first
                const int64_t d = p.site[i].d;
                const int64_t q = f / d;
                dig[i][tid] = static_cast<uint8_t>(f - q * d);
                f = q;
            }
        } else {
            uint32_t f = static_cast<uint32_t>(F);
            for (int i = p.N - 1; i >= 0; --i) {
                const uint32_t q = div_magic32(f, p.site[i].magic);
                dig[i][tid] = static_cast<uint8_t>(f - q * static_cast<uint32_t>(p.site[i].d));
                f = q;
            }
        }
        const double2 xf = x[F];
        const double2 gf = g[F];
        double hr = 0.0, hi = 0.0;
        for (int k = 0; k < p.n_diag; ++k) {
            const DevDiag dg = p.diag[k];
            double fa = local_factor64(p, dg.opa, p.site[dg.a].tab, dig[dg.a][tid]);
            if (dg.b >= 0) fa *= local_factor64(p, dg.opb, p.site[dg.b].tab, dig[dg.b][tid]);
            const double tr = fa * (dg.wr * gf.x - dg.wi * gf.y);
            const double ti = fa * (dg.wr * gf.y + dg.wi * gf.x);
            const double th = theta[dg.param];
            hr += th * tr;
            hi += th * ti;
            const int q = dg.param - p0;
            if (q >= 0 && q < kAdjParamChunk) acc[q][tid] += tr * xf.x + ti * xf.y;
        }
        for (int c = 0; c < p.n_chan; ++c) {
            const DevChan ch = p.chan[c];
            const DevSite sa = p.site[ch.a];
            const int na = dig[ch.a][tid];
            if (na - ch.qa < 0 || na - ch.qa >= sa.d) continue;  // source digit admissible (Eq. src_digit)
            double fa = local_factor64(p, ch.opa, sa.tab, na);
            if (ch.b >= 0) {
                const DevSite sb = p.site[ch.b];
                const int nb = dig[ch.b][tid];
                if (nb - ch.qb < 0 || nb - ch.qb >= sb.d) continue;
                fa *= local_factor64(p, ch.opb, sb.tab, nb);
            }
            const double2 gs = g[F - ch.delta];  // Eq. sourceoffset
            const double tr = fa * (ch.wr * gs.x - ch.wi * gs.y);
            const double ti = fa * (ch.wr * gs.y + ch.wi * gs.x);
            const double th = theta[ch.param];
            hr += th * tr;
            hi += th * ti;
            const int q = ch.param - p0;
            if (q >= 0 && q < kAdjParamChunk) acc[q][tid] += tr * xf.x + ti * xf.y;
        }
        if (write_gx) gx[F] = make_double2(hr, hi);
    }
    __syncthreads();
    const int np = p.n_params - p0 < kAdjParamChunk ? p.n_params - p0 : kAdjParamChunk;
    if (tid < np) {
        // thread q sums its parameter's column starting at column q (a rotation that keeps the threads
        // on different LDS banks); the order is fixed, so the result is deterministic
        double s = 0.0;
        for (int k = 0; k < kAdjBlock; ++k) s += acc[tid][(k + tid) & (kAdjBlock - 1)];
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
    if (!plan || !d_ws || !d_x || !d_g || !d_grad_x || !d_scratch) return MRMF_E_INVALID_ARG;
    if (plan->n_params > 0 && (!d_theta || !d_grad_theta)) return MRMF_E_INVALID_ARG;
    if (!plan->hermitian) return MRMF_E_NOT_HERMITIAN;
    if (!aligned(d_ws, 256) || !aligned(d_x, 16) || !aligned(d_g, 16) || !aligned(d_grad_x, 16) ||
        !aligned(d_scratch, 8))
        return MRMF_E_INVALID_ARG;
    const size_t vb = size_t(plan->D) * 16;
    if (ranges_overlap(d_g, vb, d_grad_x, vb) || ranges_overlap(d_x, vb, d_grad_x, vb)) return MRMF_E_INVALID_ARG;
    size_t need = 0;
    mrmf_adjoint_scratch_bytes(plan, &need);
    if (scratch_bytes < need) return MRMF_E_WORKSPACE;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const PlanArgs a = plan_args(plan, d_ws);
    const int grid = adjoint_grid(plan->D);
    double* partial = static_cast<double*>(d_scratch);
    const double* theta = plan->n_params > 0 ? d_theta : partial;  // never read when there are no params
    const int passes = plan->n_params > 0 ? (plan->n_params + kAdjParamChunk - 1) / kAdjParamChunk : 1;
    const bool wide = plan->D > int64_t(0xffffffffu);
    for (int k = 0; k < passes; ++k) {
        if (wide)
            hipLaunchKernelGGL(k_adjoint<true>, dim3(grid), dim3(kAdjBlock), 0, s, a, theta,
                               static_cast<const double2*>(d_x), static_cast<const double2*>(d_g),
                               static_cast<double2*>(d_grad_x), k * kAdjParamChunk, partial);
        else
            hipLaunchKernelGGL(k_adjoint<false>, dim3(grid), dim3(kAdjBlock), 0, s, a, theta,
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

}  // extern "C"
