// Generic gather matvec y = H x (Sec. II target-driven form): one thread per output row F, no write
// conflicts.  For each row the digits are decoded by the mixed-radix rule (Sec. III, Eq. decode), the
// diagonal terms give one weight on x_F, and every off-diagonal channel either is rejected by the
// admissibility test on its source digits or reads x at the fixed offset F - Delta (Eqs.
// src_digit_two_site, sourceoffset) with the coefficient taken from the closed-form ladder tables
// (App. A Lambda, App. B, App. C).
//
// This kernel reads everything from the uploaded plan at run time, so it serves any Hamiltonian; the
// digits of the thread's row are kept in LDS (one byte per site per thread).
#include "gersh.h"
#include "mrmf_internal.h"

namespace mrmf {

// floor(n / d) for n < 2^32 with magic = ceil(2^64 / d)
__device__ __forceinline__ uint32_t div_magic(uint32_t n, uint64_t magic) {
    return static_cast<uint32_t>(__umul64hi(magic, static_cast<uint64_t>(n)));
}

// Matrix element <n|O|n - q> of a local operator at target digit n (admissible n assumed).
template <typename R>
__device__ __forceinline__ R local_factor(const PlanArgs& p, int op, int tab, int n) {
    switch (op) {
        case MRMF_OP_Z: return static_cast<R>(p.val[tab + n]);
        case MRMF_OP_Z2: {
            const R v = static_cast<R>(p.val[tab + n]);
            return v * v;
        }
        case MRMF_OP_RAISE: return static_cast<R>(p.up[tab + n]);
        case MRMF_OP_LOWER: return static_cast<R>(p.up[tab + n + 1]);
        case MRMF_OP_RAISE2: return static_cast<R>(p.up[tab + n] * p.up[tab + n - 1]);
        case MRMF_OP_LOWER2: return static_cast<R>(p.up[tab + n + 1] * p.up[tab + n + 2]);
        default: return static_cast<R>(p.up[p.lofs[op - MRMF_OP_LOCAL_BASE] + n]);  // general one-site operator
    }
}

constexpr int kGenericBlock = 256;

template <typename R, bool WIDE>
__global__ __launch_bounds__(kGenericBlock) void k_matvec_generic(
    PlanArgs p, const R* __restrict__ theta, const typename Cx<R>::T* __restrict__ x,
    typename Cx<R>::T* __restrict__ y, const int32_t* __restrict__ skip) {
    using C = typename Cx<R>::T;
    if (skip != nullptr && *skip != 0) return;
    __shared__ uint8_t dig[kMaxSites][kGenericBlock];
    const int tid = threadIdx.x;
    const int64_t stride = int64_t(gridDim.x) * kGenericBlock;
    for (int64_t F = int64_t(blockIdx.x) * kGenericBlock + tid; F < p.D; F += stride) {
        if (WIDE) {
            int64_t f = F;
            for (int i = p.N - 1; i >= 0; --i) {
                const int64_t d = p.site[i].d;
                const int64_t q = f / d;
                dig[i][tid] = static_cast<uint8_t>(f - q * d);
                f = q;
            }
        } else {
            uint32_t f = static_cast<uint32_t>(F);
            for (int i = p.N - 1; i >= 0; --i) {
                const uint32_t q = div_magic(f, p.site[i].magic);
                dig[i][tid] = static_cast<uint8_t>(f - q * static_cast<uint32_t>(p.site[i].d));
                f = q;
            }
        }
        // diagonal weight (S_z, (S_z)^2, n, S_z S_z ...): source index is F itself
        R dr = 0, di = 0;
        for (int k = 0; k < p.n_diag; ++k) {
            const DevDiag g = p.diag[k];
            R f = local_factor<R>(p, g.opa, p.site[g.a].tab, dig[g.a][tid]);
            if (g.b >= 0) f *= local_factor<R>(p, g.opb, p.site[g.b].tab, dig[g.b][tid]);
            const R th = theta[g.param];
            dr += th * static_cast<R>(g.wr) * f;
            di += th * static_cast<R>(g.wi) * f;
        }
        const C xf = x[F];
        R ar = dr * xf.x - di * xf.y;
        R ai = dr * xf.y + di * xf.x;
        // off-diagonal channels: admissibility on the source digits, then x at F - Delta
        for (int c = 0; c < p.n_chan; ++c) {
            const DevChan ch = p.chan[c];
            const DevSite sa = p.site[ch.a];
            const int na = dig[ch.a][tid];
            const int sna = na - ch.qa;
            if (sna < 0 || sna >= sa.d) continue;
            R f = local_factor<R>(p, ch.opa, sa.tab, na);
            if (ch.b >= 0) {
                const DevSite sb = p.site[ch.b];
                const int nb = dig[ch.b][tid];
                const int snb = nb - ch.qb;
                if (snb < 0 || snb >= sb.d) continue;
                f *= local_factor<R>(p, ch.opb, sb.tab, nb);
            }
            const R th = theta[ch.param] * f;
            const R cr = th * static_cast<R>(ch.wr), ci = th * static_cast<R>(ch.wi);
            const C xs = x[F - ch.delta];
            ar += cr * xs.x - ci * xs.y;
            ai += cr * xs.y + ci * xs.x;
        }
        C out;
        out.x = ar;
        out.y = ai;
        y[F] = out;
    }
}

// Gershgorin discs of H(theta): every eigenvalue lies in some [H_FF - R_F, H_FF + R_F] with R_F the sum of
// |H_FF'| over the other entries of row F.  Per row: the diagonal (real for a Hermitian plan) from the
// diagonal terms, and for R_F the sum over the admissible channels of |theta_p w f| (at least the row's
// off-diagonal sum, several channels may meet in one entry).  Each block writes the minimum of
// H_FF - R_F and the maximum of H_FF + R_F over its rows to partial[2 b], partial[2 b + 1].
//
// TAB: every term's contribution as a function of its (one or two) digits is tabulated in LDS when the
// block starts (diagonal terms: theta_p w_r f_a(n_a) f_b(n_b); channels: |theta_p w f_a(n_a) f_b(n_b)|, 0
// where a source digit leaves its range), so that a row costs one LDS read per term; the tables of all
// terms together must fit kGershTab entries.  Without TAB the row evaluates the factors itself.
constexpr int kGershTab = 2048;
constexpr int kGershMaxTerms = 256;

template <bool WIDE, bool TAB>
__global__ __launch_bounds__(kGenericBlock) void k_gershgorin(PlanArgs p, const double* __restrict__ theta,
                                                               double* __restrict__ partial) {
    __shared__ uint8_t dig[kMaxSites][kGenericBlock];
    __shared__ double slo[kGenericBlock], shi[kGenericBlock];
    __shared__ double tab[TAB ? kGershTab : 1];
    __shared__ int4 td[TAB ? kGershMaxTerms : 1];  // per term: site a, site b (-1: none), d_b (1), table offset
    const int tid = threadIdx.x;
    const int nt = p.n_diag + p.n_chan;
    if constexpr (TAB) {
        if (tid == 0) {  // table offsets, diagonal terms first (the host checked that they fit)
            int off = 0;
            for (int k = 0; k < nt; ++k) {
                const bool dg = k < p.n_diag;
                const int ta = dg ? p.diag[k].a : p.chan[k - p.n_diag].a;
                const int tb = dg ? p.diag[k].b : p.chan[k - p.n_diag].b;
                const int db = tb >= 0 ? p.site[tb].d : 1;
                td[k] = make_int4(ta, tb, db, off);
                off += p.site[ta].d * db;
            }
        }
        __syncthreads();
        for (int k = 0; k < nt; ++k) {
            const int4 t = td[k];
            const int n = p.site[t.x].d * t.z;
            for (int e = tid; e < n; e += kGenericBlock) {
                const int na = e / t.z, nb = e - na * t.z;
                double v;
                if (k < p.n_diag) {
                    const DevDiag g = p.diag[k];
                    double f = local_factor<double>(p, g.opa, p.site[g.a].tab, na);
                    if (g.b >= 0) f *= local_factor<double>(p, g.opb, p.site[g.b].tab, nb);
                    v = theta[g.param] * g.wr * f;
                } else {
                    const DevChan ch = p.chan[k - p.n_diag];
                    bool ok = na - ch.qa >= 0 && na - ch.qa < p.site[ch.a].d;
                    double f = local_factor<double>(p, ch.opa, p.site[ch.a].tab, na);
                    if (ch.b >= 0) {
                        ok = ok && nb - ch.qb >= 0 && nb - ch.qb < p.site[ch.b].d;
                        f *= local_factor<double>(p, ch.opb, p.site[ch.b].tab, nb);
                    }
                    v = ok ? fabs(theta[ch.param] * f) * sqrt(ch.wr * ch.wr + ch.wi * ch.wi) : 0.0;
                }
                tab[t.w + e] = v;
            }
        }
        __syncthreads();
    }
    double lo = __builtin_inf(), hi = -__builtin_inf();
    const int64_t stride = int64_t(gridDim.x) * kGenericBlock;
    for (int64_t F = int64_t(blockIdx.x) * kGenericBlock + tid; F < p.D; F += stride) {
        if (WIDE) {
            int64_t f = F;
            for (int i = p.N - 1; i >= 0; --i) {
                const int64_t d = p.site[i].d;
                const int64_t q = f / d;
                dig[i][tid] = static_cast<uint8_t>(f - q * d);
                f = q;
            }
        } else {
            uint32_t f = static_cast<uint32_t>(F);
            for (int i = p.N - 1; i >= 0; --i) {
                const uint32_t q = div_magic(f, p.site[i].magic);
                dig[i][tid] = static_cast<uint8_t>(f - q * static_cast<uint32_t>(p.site[i].d));
                f = q;
            }
        }
        double diag = 0.0, rad = 0.0;
        if constexpr (TAB) {
            for (int k = 0; k < nt; ++k) {
                const int4 t = td[k];
                const int e = dig[t.x][tid] * t.z + (t.y >= 0 ? dig[t.y][tid] : 0);
                if (k < p.n_diag)
                    diag += tab[t.w + e];
                else
                    rad += tab[t.w + e];
            }
        } else {
            for (int k = 0; k < p.n_diag; ++k) {
                const DevDiag g = p.diag[k];
                double fa = local_factor<double>(p, g.opa, p.site[g.a].tab, dig[g.a][tid]);
                if (g.b >= 0) fa *= local_factor<double>(p, g.opb, p.site[g.b].tab, dig[g.b][tid]);
                diag += theta[g.param] * g.wr * fa;
            }
            for (int c = 0; c < p.n_chan; ++c) {
                const DevChan ch = p.chan[c];
                const DevSite sa = p.site[ch.a];
                const int na = dig[ch.a][tid];
                if (na - ch.qa < 0 || na - ch.qa >= sa.d) continue;
                double fa = local_factor<double>(p, ch.opa, sa.tab, na);
                if (ch.b >= 0) {
                    const DevSite sb = p.site[ch.b];
                    const int nb = dig[ch.b][tid];
                    if (nb - ch.qb < 0 || nb - ch.qb >= sb.d) continue;
                    fa *= local_factor<double>(p, ch.opb, sb.tab, nb);
                }
                rad += fabs(theta[ch.param] * fa) * sqrt(ch.wr * ch.wr + ch.wi * ch.wi);
            }
        }
        lo = fmin(lo, diag - rad);
        hi = fmax(hi, diag + rad);
    }
    slo[tid] = lo;
    shi[tid] = hi;
    __syncthreads();
    if (tid == 0) {
        for (int k = 1; k < kGenericBlock; ++k) {
            lo = fmin(lo, slo[k]);
            hi = fmax(hi, shi[k]);
        }
        partial[2 * blockIdx.x] = lo;
        partial[2 * blockIdx.x + 1] = hi;
    }
}

// The same ends over count coupling vectors theta + s * stride in one pass (linear form of gersh.h).
template <bool WIDE>
__global__ __launch_bounds__(kGenericBlock) void k_gershgorin_lin(PlanArgs p, const double* __restrict__ theta,
                                                                   int64_t stride, int32_t count,
                                                                   double* __restrict__ partial) {
    static_assert(kGenericBlock == kLinBlock, "block size of the shared bounds code");
    __shared__ GershLinLds L;
    __shared__ uint8_t dig[kMaxSites][kGenericBlock];
    __shared__ double slo[kGenericBlock], shi[kGenericBlock];
    const int tid = threadIdx.x;
    gersh_lin_tables(p, [&](int op, int tab, int n) { return local_factor<double>(p, op, tab, n); }, L);
    double lo = __builtin_inf(), hi = -__builtin_inf();
    const int64_t step = int64_t(gridDim.x) * kGenericBlock;
    for (int64_t F = int64_t(blockIdx.x) * kGenericBlock + tid; F < p.D; F += step) {
        if (WIDE) {
            int64_t f = F;
            for (int i = p.N - 1; i >= 0; --i) {
                const int64_t d = p.site[i].d;
                const int64_t q = f / d;
                dig[i][tid] = static_cast<uint8_t>(f - q * d);
                f = q;
            }
        } else {
            uint32_t f = static_cast<uint32_t>(F);
            for (int i = p.N - 1; i >= 0; --i) {
                const uint32_t q = div_magic(f, p.site[i].magic);
                dig[i][tid] = static_cast<uint8_t>(f - q * static_cast<uint32_t>(p.site[i].d));
                f = q;
            }
        }
        gersh_lin_row(p, L, dig, theta, stride, count, lo, hi);
    }
    gersh_block_ends(lo, hi, slo, shi, partial);
}

__global__ __launch_bounds__(kLinBlock) void k_gershgorin_finalize(const double* __restrict__ partial, int nb,
                                                        double* __restrict__ out) {
    gersh_finalize_block(partial, nb, out);
}

constexpr int kGershMaxGrid = 1024;

inline int gershgorin_grid(int64_t D) {
    const int64_t b = (D + kGenericBlock - 1) / kGenericBlock;
    return static_cast<int>(b < kGershMaxGrid ? b : kGershMaxGrid);
}

__global__ __launch_bounds__(kGenericBlock) void k_debug_sources(PlanArgs p, int64_t F0, int64_t count,
                                                                 int64_t* __restrict__ out) {
    const int64_t r = int64_t(blockIdx.x) * kGenericBlock + threadIdx.x;
    if (r >= count) return;
    const int64_t F = F0 + r;
    for (int c = 0; c < p.n_chan; ++c) {
        const DevChan ch = p.chan[c];
        const int64_t da = p.site[ch.a].d;
        const int na = static_cast<int>((F / p.site[ch.a].M) % da);
        bool ok = na - ch.qa >= 0 && na - ch.qa < da;
        if (ch.b >= 0) {
            const int64_t db = p.site[ch.b].d;
            const int nb = static_cast<int>((F / p.site[ch.b].M) % db);
            ok = ok && nb - ch.qb >= 0 && nb - ch.qb < db;
        }
        out[r * p.n_chan + c] = ok ? F - ch.delta : -1;
    }
}

namespace {

int generic_grid(int64_t D) {
    const int64_t blocks = (D + kGenericBlock - 1) / kGenericBlock;
    return static_cast<int>(blocks < 262144 ? blocks : 262144);
}

template <typename R>
mrmf_status matvec_dispatch(mrmf_plan_t* p, const void* d_ws, const R* theta, const void* x, void* y,
                            hipStream_t s, const int32_t* d_skip) {
    using C = typename Cx<R>::T;
    if (!p || !d_ws || !theta || !x || !y) return MRMF_E_INVALID_ARG;
    if (!aligned(d_ws, 256) || !aligned(x, sizeof(C)) || !aligned(y, sizeof(C))) return MRMF_E_INVALID_ARG;
    const size_t bytes = size_t(p->D) * sizeof(C);
    if (ranges_overlap(x, bytes, y, bytes)) return MRMF_E_INVALID_ARG;
    const int dtype = sizeof(R) == 4 ? MRMF_DTYPE_C : MRMF_DTYPE_Z;
    const int32_t mode = p->cfg[dtype].mode;
    if (mode != MRMF_KERNEL_GENERIC) {
        const mrmf_status st = spec_launch(p, dtype, theta, x, y, s, d_skip);
        if (st == MRMF_OK || !(st == MRMF_E_UNSUPPORTED && mode == MRMF_KERNEL_AUTO)) return st;
    }
    const PlanArgs a = plan_args(p, d_ws);
    const int grid = generic_grid(p->D);
    if (p->D <= int64_t(0xffffffffu))
        hipLaunchKernelGGL((k_matvec_generic<R, false>), dim3(grid), dim3(kGenericBlock), 0, s, a, theta,
                           static_cast<const C*>(x), static_cast<C*>(y), d_skip);
    else
        hipLaunchKernelGGL((k_matvec_generic<R, true>), dim3(grid), dim3(kGenericBlock), 0, s, a, theta,
                           static_cast<const C*>(x), static_cast<C*>(y), d_skip);
    return launch_status();
}

}  // namespace

mrmf_status matvec_z_impl(mrmf_plan_t* p, const void* d_ws, const double* theta, const void* x, void* y,
                          hipStream_t s, const int32_t* d_skip) {
    return matvec_dispatch<double>(p, d_ws, theta, x, y, s, d_skip);
}

mrmf_status matvec_c_impl(mrmf_plan_t* p, const void* d_ws, const float* theta, const void* x, void* y,
                          hipStream_t s, const int32_t* d_skip) {
    return matvec_dispatch<float>(p, d_ws, theta, x, y, s, d_skip);
}

}  // namespace mrmf

extern "C" {

mrmf_status mrmf_matvec_z(mrmf_plan plan, const void* d_ws, const double* d_theta, const void* d_x,
                          void* d_y, mrmf_stream stream) {
    return mrmf::matvec_z_impl(plan, d_ws, d_theta, d_x, d_y, static_cast<hipStream_t>(stream), nullptr);
}

mrmf_status mrmf_matvec_c(mrmf_plan plan, const void* d_ws, const float* d_theta, const void* d_x,
                          void* d_y, mrmf_stream stream) {
    return mrmf::matvec_c_impl(plan, d_ws, d_theta, d_x, d_y, static_cast<hipStream_t>(stream), nullptr);
}

mrmf_status mrmf_debug_sources(mrmf_plan plan, const void* d_ws, int64_t F0, int64_t count,
                               int64_t* d_out, mrmf_stream stream) {
    if (!plan || !d_ws || !d_out || F0 < 0 || count < 0 || F0 > plan->D - count) return MRMF_E_INVALID_ARG;
    if (count == 0 || plan->chans.empty()) return MRMF_OK;
    const mrmf::PlanArgs a = mrmf::plan_args(plan, d_ws);
    const int64_t blocks = (count + mrmf::kGenericBlock - 1) / mrmf::kGenericBlock;
    if (blocks > 0x7fffffff) return MRMF_E_INVALID_ARG;
    hipLaunchKernelGGL(mrmf::k_debug_sources, dim3(static_cast<unsigned>(blocks)), dim3(mrmf::kGenericBlock), 0,
                       static_cast<hipStream_t>(stream), a, F0, count, d_out);
    return mrmf::launch_status();
}

mrmf_status mrmf_spectral_bounds_scratch_bytes(mrmf_plan plan, size_t* bytes) {
    if (!plan || !bytes) return MRMF_E_INVALID_ARG;
    *bytes = sizeof(double) * 2 * size_t(mrmf::gershgorin_grid(plan->D));
    return MRMF_OK;
}

mrmf_status mrmf_spectral_bounds(mrmf_plan plan, const void* d_ws, const double* d_theta, double* d_out,
                                 void* d_scratch, size_t scratch_bytes, mrmf_stream stream) {
    using namespace mrmf;
    if (!plan || !d_ws || !d_out || !d_scratch || (plan->n_params > 0 && !d_theta)) return MRMF_E_INVALID_ARG;
    if (!plan->hermitian) return MRMF_E_NOT_HERMITIAN;
    if (!aligned(d_ws, 256) || !aligned(d_scratch, 8) || !aligned(d_out, 8)) return MRMF_E_INVALID_ARG;
    size_t need = 0;
    mrmf_spectral_bounds_scratch_bytes(plan, &need);
    if (scratch_bytes < need) return MRMF_E_WORKSPACE;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int grid = gershgorin_grid(plan->D);
    double* partial = static_cast<double*>(d_scratch);
    const double* theta = plan->n_params > 0 ? d_theta : partial;  // never read when there are no params
    // per-term digit tables in LDS when they fit
    const int nt = static_cast<int>(plan->diags.size() + plan->chans.size());
    int64_t entries = 0;
    for (const auto& g : plan->diags) entries += int64_t(plan->d[g.a]) * (g.b >= 0 ? plan->d[g.b] : 1);
    for (const auto& c : plan->chans) entries += int64_t(plan->d[c.a]) * (c.b >= 0 ? plan->d[c.b] : 1);
    const bool tab = nt <= kGershMaxTerms && entries <= kGershTab;
    const bool narrow = plan->D <= int64_t(0xffffffffu);
    const dim3 g(grid), b(kGenericBlock);
    const PlanArgs pa = plan_args(plan, d_ws);
    if (narrow && tab) hipLaunchKernelGGL((k_gershgorin<false, true>), g, b, 0, s, pa, theta, partial);
    else if (narrow) hipLaunchKernelGGL((k_gershgorin<false, false>), g, b, 0, s, pa, theta, partial);
    else if (tab) hipLaunchKernelGGL((k_gershgorin<true, true>), g, b, 0, s, pa, theta, partial);
    else hipLaunchKernelGGL((k_gershgorin<true, false>), g, b, 0, s, pa, theta, partial);
    hipLaunchKernelGGL(k_gershgorin_finalize, dim3(1), dim3(kLinBlock), 0, s, partial, grid, d_out);
    return launch_status();
}

mrmf_status mrmf_spectral_bounds_many(mrmf_plan plan, const void* d_ws, const double* d_theta, int64_t theta_stride,
                                      int32_t count, double* d_out, void* d_scratch, size_t scratch_bytes,
                                      mrmf_stream stream) {
    using namespace mrmf;
    if (!plan || !d_ws || !d_out || !d_scratch || (plan->n_params > 0 && !d_theta) || count < 1 ||
        theta_stride < 0)
        return MRMF_E_INVALID_ARG;
    if (!plan->hermitian) return MRMF_E_NOT_HERMITIAN;
    if (!aligned(d_ws, 256) || !aligned(d_scratch, 8) || !aligned(d_out, 8)) return MRMF_E_INVALID_ARG;
    size_t need = 0;
    mrmf_spectral_bounds_scratch_bytes(plan, &need);
    if (scratch_bytes < need) return MRMF_E_WORKSPACE;
    if (!gersh_lin_fits(plan->n_params, plan->d, plan->diags, plan->chans)) return MRMF_E_UNSUPPORTED;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int grid = gershgorin_grid(plan->D);
    double* partial = static_cast<double*>(d_scratch);
    const double* theta = plan->n_params > 0 ? d_theta : partial;  // never read when there are no params
    if (plan->D <= int64_t(0xffffffffu))
        hipLaunchKernelGGL(k_gershgorin_lin<false>, dim3(grid), dim3(kGenericBlock), 0, s, plan_args(plan, d_ws),
                           theta, theta_stride, count, partial);
    else
        hipLaunchKernelGGL(k_gershgorin_lin<true>, dim3(grid), dim3(kGenericBlock), 0, s, plan_args(plan, d_ws),
                           theta, theta_stride, count, partial);
    hipLaunchKernelGGL(k_gershgorin_finalize, dim3(1), dim3(kLinBlock), 0, s, partial, grid, d_out);
    return launch_status();
}

}  // extern "C"
