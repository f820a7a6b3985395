// Device-resident Lanczos eigensolver driving the matrix-free map (the Krylov use of x -> H x, Sec. I)
// and the FP64 vector reductions it needs.  Every scalar of the recurrence (alpha_j, beta_j, the Gram-
// Schmidt coefficients, the Ritz value) stays in device memory; the host only enqueues kernels.  After a
// breakdown every later kernel of the call sees the `stopped` flag and returns at once.
#include <cmath>
#include <cstddef>

#include "mrmf_internal.h"
#include "reduce.h"

namespace mrmf {
namespace {

constexpr int kRB = 256;            // threads per reduction block
constexpr int kMaxRedBlocks = 512;  // first-stage partials per reduction
constexpr int kGroup = 8;           // basis vectors per Gram-Schmidt block

struct LzState {
    int32_t stopped;  // recurrence ended (breakdown, zero start vector, or last step done)
    int32_t steps;    // k: number of alpha_j computed
    int32_t breakdown;
    int32_t skip2;    // conditional Gram-Schmidt: the second pass of this step is skipped (or stopped)
    double tnorm;  // Gershgorin estimate of ||T|| so far
    double nrm0;   // ||v0||
    double theta;  // lowest Ritz value
    double wn2;    // conditional Gram-Schmidt: ||w||^2 before the first pass
    int32_t n_second;  // conditional Gram-Schmidt: second passes taken so far
    int32_t n_pro;     // partial reorthogonalisation: full Gram-Schmidt passes taken so far
    int32_t skip_pro;  // partial reorthogonalisation: this step's pass (and its norm) is skipped
    int32_t force;     // partial reorthogonalisation: the next step reorthogonalises as well
    double unrm;       // ||V s|| of the Ritz vector before it is normalised
    int32_t skip_u;    // the Ritz vector is zero (no step taken): left as it is
    int32_t pad;
};

int red_blocks(int64_t n) {
    const int64_t b = (n + kRB - 1) / kRB;
    return static_cast<int>(b < kMaxRedBlocks ? (b < 1 ? 1 : b) : kMaxRedBlocks);
}

__device__ __forceinline__ bool halted(const int32_t* stopped) { return stopped != nullptr && *stopped != 0; }

// ---------------------------------------------------------------- first-stage reductions
__global__ __launch_bounds__(kRB) void k_norm2_partial(int64_t n, const double2* __restrict__ a,
                                                        double* __restrict__ partial,
                                                        const int32_t* __restrict__ stopped) {
    if (halted(stopped)) return;
    __shared__ double lds[kRB / 64];
    double v[1] = {0.0};
    for (int64_t i = int64_t(blockIdx.x) * kRB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kRB) {
        const double2 x = a[i];
        v[0] += x.x * x.x + x.y * x.y;
    }
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = v[0];
}

// partial[b] = sum over the block's rows of conj(a) b
__global__ __launch_bounds__(kRB) void k_dot_partial(int64_t n, const double2* __restrict__ a,
                                                      const double2* __restrict__ b,
                                                      double2* __restrict__ partial,
                                                      const int32_t* __restrict__ stopped) {
    if (halted(stopped)) return;
    __shared__ double lds[2 * kRB / 64];
    double v[2] = {0.0, 0.0};
    for (int64_t i = int64_t(blockIdx.x) * kRB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kRB) {
        const double2 x = a[i], y = b[i];
        v[0] += x.x * y.x + x.y * y.y;
        v[1] += x.x * y.y - x.y * y.x;
    }
    block_sum<2>(v, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = make_double2(v[0], v[1]);
}

// partial[b] = sum over the block's rows of conj(a) b for a c64 b (the c64 matvec's output, read as it is)
__global__ __launch_bounds__(kRB) void k_dot_partial32(int64_t n, const double2* __restrict__ a,
                                                        const float2* __restrict__ b,
                                                        double2* __restrict__ partial,
                                                        const int32_t* __restrict__ stopped) {
    if (halted(stopped)) return;
    __shared__ double lds[2 * kRB / 64];
    double v[2] = {0.0, 0.0};
    for (int64_t i = int64_t(blockIdx.x) * kRB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kRB) {
        const double2 x = a[i];
        const float2 y = b[i];
        v[0] += x.x * static_cast<double>(y.x) + x.y * static_cast<double>(y.y);
        v[1] += x.x * static_cast<double>(y.y) - x.y * static_cast<double>(y.x);
    }
    block_sum<2>(v, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = make_double2(v[0], v[1]);
}

// ||hu - theta u||^2 partials
__global__ __launch_bounds__(kRB) void k_resid_partial(int64_t n, const double2* __restrict__ hu,
                                                        const double2* __restrict__ u,
                                                        const LzState* __restrict__ st,
                                                        double* __restrict__ partial) {
    __shared__ double lds[kRB / 64];
    double v[1] = {0.0};
    const double th = st->theta;
    for (int64_t i = int64_t(blockIdx.x) * kRB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kRB) {
        const double2 a = hu[i], b = u[i];
        const double rx = a.x - th * b.x, ry = a.y - th * b.y;
        v[0] += rx * rx + ry * ry;
    }
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = v[0];
}

// Gram-Schmidt coefficients c_i = <V_i|w>, i = 0..k-1: partial[i * nb + block]
__global__ __launch_bounds__(kRB) void k_gemvt_partial(int64_t n, const double2* __restrict__ V, int k,
                                                        const double2* __restrict__ w,
                                                        double2* __restrict__ partial, int nb,
                                                        const int32_t* __restrict__ stopped) {
    if (halted(stopped)) return;
    __shared__ double lds[2 * kGroup * kRB / 64];
    const int base = blockIdx.y * kGroup;
    double v[2 * kGroup];
#pragma unroll
    for (int g = 0; g < 2 * kGroup; ++g) v[g] = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kRB + threadIdx.x; i < n; i += int64_t(nb) * kRB) {
        const double2 y = w[i];
#pragma unroll
        for (int g = 0; g < kGroup; ++g) {
            if (base + g < k) {
                const double2 x = V[int64_t(base + g) * n + i];
                v[2 * g] += x.x * y.x + x.y * y.y;
                v[2 * g + 1] += x.x * y.y - x.y * y.x;
            }
        }
    }
    block_sum<2 * kGroup>(v, lds);
    if (threadIdx.x == 0) {
        for (int g = 0; g < kGroup; ++g)
            if (base + g < k) partial[int64_t(base + g) * nb + blockIdx.x] = make_double2(v[2 * g], v[2 * g + 1]);
    }
}

__global__ void k_gemvt_finalize(int k, int nb, const double2* __restrict__ partial, double2* __restrict__ c,
                                 const int32_t* __restrict__ stopped) {
    if (halted(stopped)) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k) return;
    double sr = 0.0, si = 0.0;
    for (int b = 0; b < nb; ++b) {
        sr += partial[int64_t(i) * nb + b].x;
        si += partial[int64_t(i) * nb + b].y;
    }
    c[i] = make_double2(sr, si);
}

// w = (zero ? 0 : w) + sgn * sum_{i<k} c_i V_i  (k read from kdev when given)
__global__ __launch_bounds__(kRB) void k_gemv_acc(int64_t n, const double2* __restrict__ V, int k,
                                                   const int32_t* __restrict__ kdev,
                                                   const double2* __restrict__ c, double2* __restrict__ w,
                                                   int zero, double sgn, const int32_t* __restrict__ stopped) {
    if (halted(stopped)) return;
    const int kk = kdev ? *kdev : k;
    for (int64_t i = int64_t(blockIdx.x) * kRB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kRB) {
        double ar = 0.0, ai = 0.0;
        for (int g = 0; g < kk; ++g) {
            const double2 cg = c[g], x = V[int64_t(g) * n + i];
            ar += cg.x * x.x - cg.y * x.y;
            ai += cg.x * x.y + cg.y * x.x;
        }
        if (zero) {
            w[i] = make_double2(sgn * ar, sgn * ai);
        } else {
            const double2 y = w[i];
            w[i] = make_double2(y.x + sgn * ar, y.y + sgn * ai);
        }
    }
}

// w = (h32 ? h32 upcast : w) - alpha v_j - beta v_{j-1}, and the partial sums of ||w||^2 (one per block;
// launched with the reduction grid, so the partials are those k_norm2_partial would give)
__global__ __launch_bounds__(kRB) void k_three_term_norm(int64_t n, double2* __restrict__ w,
                                                          const float2* __restrict__ h32,
                                                          const double2* __restrict__ vj,
                                                          const double2* __restrict__ vjm1,
                                                          const double* __restrict__ alpha,
                                                          const double* __restrict__ beta,
                                                          double* __restrict__ partial,
                                                          const int32_t* __restrict__ stopped) {
    if (halted(stopped)) return;
    __shared__ double lds[kRB / 64];
    const double a = *alpha;
    const double b = vjm1 ? *beta : 0.0;
    double v[1] = {0.0};
    for (int64_t i = int64_t(blockIdx.x) * kRB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kRB) {
        double2 y;
        if (h32) {
            const float2 h = h32[i];
            y = make_double2(h.x, h.y);
        } else {
            y = w[i];
        }
        const double2 x = vj[i];
        y.x -= a * x.x;
        y.y -= a * x.y;
        if (vjm1) {
            const double2 z = vjm1[i];
            y.x -= b * z.x;
            y.y -= b * z.y;
        }
        w[i] = y;
        v[0] += y.x * y.x + y.y * y.y;
    }
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = v[0];
}

// dst = src / denom (and a c64 copy when dst32 is given)
__global__ __launch_bounds__(kRB) void k_scale(int64_t n, const double2* src, double2* dst,
                                                const double* __restrict__ denom, float2* __restrict__ dst32,
                                                const int32_t* __restrict__ stopped) {
    if (halted(stopped)) return;
    const double s = *denom;
    for (int64_t i = int64_t(blockIdx.x) * kRB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kRB) {
        const double2 x = src[i];
        const double2 y = make_double2(x.x / s, x.y / s);
        dst[i] = y;
        if (dst32) dst32[i] = make_float2(static_cast<float>(y.x), static_cast<float>(y.y));
    }
}

// ---------------------------------------------------------------- second stages
__global__ void k_init_finalize(const double* __restrict__ partial, int nb, LzState* __restrict__ st) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partial[b];
    const double nrm = sqrt(s);
    st->steps = 0;
    st->breakdown = 0;
    st->skip2 = 0;
    st->wn2 = 0.0;
    st->n_second = 0;
    st->n_pro = 0;
    st->skip_pro = 1;
    st->force = 0;
    st->tnorm = 0.0;
    st->nrm0 = nrm;
    st->theta = __builtin_nan("");
    st->stopped = (nrm > 0.0 && isfinite(nrm)) ? 0 : 1;
}

__global__ void k_alpha_finalize(const double2* __restrict__ partial, int nb, double* __restrict__ alpha,
                                 const int32_t* __restrict__ stopped) {
    if (halted(stopped)) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partial[b].x;
    *alpha = s;
}

// Conditional Gram-Schmidt: wn2 = ||w||^2 before the first pass (store = 1), or after it (store = 0):
// skip2 = 1 unless the pass shrank ||w||^2 below half (or the recurrence has stopped).
__global__ void k_cgs_norm(const double* __restrict__ partial, int nb, int store, LzState* __restrict__ st) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partial[b];
    if (store) {
        st->wn2 = s;
        return;
    }
    const int skip = st->stopped != 0 || s >= 0.5 * st->wn2;
    st->skip2 = skip;
    if (!skip) ++st->n_second;
}

// Partial reorthogonalisation (H. D. Simon, "The Lanczos algorithm with partial reorthogonalization",
// Math. Comp. 42 (1984)): the inner products omega_{i,k} = <v_i|v_k> are not computed but estimated from
// the recurrence that the Lanczos relation beta_j v_{j+1} = H v_j - alpha_j v_j - beta_{j-1} v_{j-1}
// implies for them,
//     beta_j omega_{j+1,k} = beta_k omega_{j,k+1} + (alpha_k - alpha_j) omega_{j,k} + beta_{k-1} omega_{j,k-1}
//                            - beta_{j-1} omega_{j-1,k},      omega_{k,k} = 1,
// with a rounding term 2 eps ||T||, of the sign that increases |omega|, added to every new estimate, and
// omega_{j+1,j} = eps64 sqrt(D) ||T|| / beta_j (the level the FP64 three-term step leaves).  eps is the
// machine epsilon of the matvec: FP64's, or FP32's for the c64 form, whose matvec error of about
// eps32 ||H|| per step is what its basis loses orthogonality to.  (A rounding term scaled down by
// 1 / sqrt(D), as for an error vector unrelated to the basis, was measured to be unsafe: on the 20-site
// ring the c64 form's basis then drifted to |<v_i|v_k>| = 0.13.)  When some estimate exceeds sqrt(eps),
// w = beta_j v_{j+1} is orthogonalised against every earlier vector (one classical Gram-Schmidt pass, in
// FP64), and so is the next step's (the loss of orthogonality spreads to it through the recurrence); the
// estimates then restart at eps64 sqrt(D).  Semi-orthogonality (every |omega| <= sqrt(eps)) keeps the
// Ritz values as accurate as full reorthogonalisation would, to O(eps ||H||).
// One block; omega rows i at omega + (i mod 3) (m + 2); partial: the ||w||^2 partial sums of this step.
__global__ __launch_bounds__(kRB) void k_pro_estimate(const double* __restrict__ partial, int nb, int j, int m,
                                                      int64_t D, double eps, const double* __restrict__ alpha,
                                                      const double* __restrict__ beta, double* __restrict__ omega,
                                                      LzState* __restrict__ st) {
    __shared__ double red[kRB];
    __shared__ double s_bj;
    const int tid = threadIdx.x;
    if (st->stopped) {
        if (tid == 0) st->skip_pro = 1;
        return;
    }
    if (tid == 0) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += partial[b];
        s_bj = sqrt(s);
    }
    __syncthreads();
    const double bj = s_bj;
    const double eps64 = 2.220446049250313e-16;
    const double tn = fmax(st->tnorm, fabs(alpha[j]) + bj + (j > 0 ? beta[j - 1] : 0.0));
    const double* wc = omega + (j % 3) * (m + 2);          // omega_{j, k}, k < j
    const double* wp = omega + ((j + 2) % 3) * (m + 2);    // omega_{j-1, k}, k < j - 1
    double* wn = omega + ((j + 1) % 3) * (m + 2);          // omega_{j+1, k}, k <= j
    const double level = eps64 * sqrt(static_cast<double>(D));
    const bool usable = bj > 0.0 && isfinite(bj);
    double mx = 0.0;
    if (usable) {
        auto oc = [&](int k) { return k == j ? 1.0 : wc[k]; };
        auto op = [&](int k) { return j == 0 ? 0.0 : (k == j - 1 ? 1.0 : wp[k]); };
        for (int k = tid; k <= j; k += kRB) {
            double t;
            if (k < j) {
                t = beta[k] * oc(k + 1) + (alpha[k] - alpha[j]) * oc(k) - (j > 0 ? beta[j - 1] * op(k) : 0.0);
                if (k > 0) t += beta[k - 1] * oc(k - 1);
                t += (t >= 0.0 ? 2.0 : -2.0) * eps * tn;
                t /= bj;
            } else {
                t = level * tn / bj;
            }
            wn[k] = t;
            mx = fmax(mx, fabs(t));
        }
    }
    red[tid] = mx;
    __syncthreads();
    for (int w = kRB / 2; w > 0; w >>= 1) {
        if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
        __syncthreads();
    }
    const bool over = usable && red[0] > sqrt(eps);
    const bool now = usable && (over || st->force != 0);
    __syncthreads();
    if (now)
        for (int k = tid; k <= j; k += kRB) wn[k] = level;
    if (tid == 0) {
        st->skip_pro = now ? 0 : 1;
        st->force = over ? 1 : 0;
        if (now) ++st->n_pro;
    }
}

__global__ void k_beta_finalize(const double* __restrict__ partial, int nb, int j, int last,
                                const double* __restrict__ alpha, double* __restrict__ beta,
                                LzState* __restrict__ st) {
    if (st->stopped) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partial[b];
    const double bj = sqrt(s);
    beta[j] = bj;
    const double t = fabs(alpha[j]) + bj + (j > 0 ? beta[j - 1] : 0.0);
    st->tnorm = fmax(st->tnorm, t);
    st->steps = j + 1;
    if (last) {
        st->stopped = 1;
    } else if (bj <= 1e-14 * st->tnorm) {
        st->stopped = 1;
        st->breakdown = 1;
    }
}

// ||V s|| of the Ritz vector (a basis that is only semi-orthogonal leaves it 1 + O(sqrt(eps))).
__global__ void k_unorm_finalize(const double* __restrict__ partial, int nb, LzState* __restrict__ st) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partial[b];
    st->unrm = sqrt(s);
    st->skip_u = (st->unrm > 0.0 && isfinite(st->unrm)) ? 0 : 1;
}

__global__ void k_scalar_finalize(const double* __restrict__ partial, int nb, double* __restrict__ out, int sq) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partial[b];
    *out = sq ? sqrt(s) : s;
}

__global__ void k_dot_finalize(const double2* __restrict__ partial, int nb, double* __restrict__ out) {
    double sr = 0.0, si = 0.0;
    for (int b = 0; b < nb; ++b) {
        sr += partial[b].x;
        si += partial[b].y;
    }
    out[0] = sr;
    out[1] = si;
}

// Number of eigenvalues of the k x k symmetric tridiagonal (a, b) below x: the count of negative pivots
// of the LDL^T factorisation of T - x I (Sturm sequence count, Sylvester's law of inertia), the basis of
// the bisection method of Barth, Martin and Wilkinson (1967); pivots below pivmin in magnitude are
// replaced by -pivmin so the recurrence never divides by zero.
__device__ int sturm_count(const double* a, const double* b, int k, double x, double pivmin) {
    int cnt = 0;
    double q = a[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0) ++cnt;
    for (int i = 1; i < k; ++i) {
        q = a[i] - x - b[i - 1] * b[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        if (q < 0) ++cnt;
    }
    return cnt;
}

// Lowest eigenpair of T (one thread; k is small): the lowest eigenvalue by bisection on the Sturm count
// (Barth, Martin and Wilkinson), then its eigenvector by inverse iteration (Wilkinson; Peters and
// Wilkinson 1971) with T - theta I factored by Gaussian elimination with partial pivoting, which for a
// tridiagonal matrix keeps a lower band of one and an upper band of two (dl, d, du, du2).
// work: 5 * m doubles.  s_out: complex coefficients (s_i, 0) for the Ritz vector, zero past k.
__global__ void k_tridiag_lowest(const double* __restrict__ alpha, const double* __restrict__ beta, int m,
                                 LzState* __restrict__ st, double* __restrict__ work,
                                 double2* __restrict__ s_out, double* __restrict__ result) {
    const int k = st->steps;
    const double qnan = __builtin_nan("");
    for (int i = 0; i < m; ++i) s_out[i] = make_double2(0.0, 0.0);
    if (k == 0) {
        result[0] = result[1] = result[2] = qnan;
        result[3] = 0.0;
        st->theta = qnan;
        return;
    }
    const double* a = alpha;
    const double* b = beta;
    double lo = INFINITY, hi = -INFINITY, bmax2 = 0.0;
    for (int i = 0; i < k; ++i) {
        const double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i < k - 1 ? fabs(b[i]) : 0.0);
        lo = fmin(lo, a[i] - r);
        hi = fmax(hi, a[i] + r);
        if (i < k - 1) bmax2 = fmax(bmax2, b[i] * b[i]);
    }
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, bmax2);
    const double tn = fmax(fabs(lo), fabs(hi));
    lo -= 4.0 * 2.220446049250313e-16 * tn + pivmin;
    hi += 4.0 * 2.220446049250313e-16 * tn + pivmin;
    for (int it = 0; it < 400; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (sturm_count(a, b, k, mid, pivmin) >= 1)
            hi = mid;
        else
            lo = mid;
    }
    const double theta = 0.5 * (lo + hi);
    // inverse iteration: LU with partial pivoting of T - theta I (rows swapped as needed)
    double* dl = work;
    double* d = work + m;
    double* du = work + 2 * m;
    double* du2 = work + 3 * m;
    double* x = work + 4 * m;
    double sn = 0.0;
    for (int i = 0; i < k; ++i) x[i] = 1.0;
    const double tiny = 2.220446049250313e-16 * fmax(tn, 1e-300);
    for (int iter = 0; iter < 3; ++iter) {
        for (int i = 0; i < k; ++i) {
            d[i] = a[i] - theta;
            if (i < k - 1) dl[i] = du[i] = b[i];
            du2[i] = 0.0;
        }
        // factor with row interchanges, applying the same eliminations to the right-hand side
        for (int i = 0; i < k - 1; ++i) {
            if (fabs(d[i]) >= fabs(dl[i])) {
                if (d[i] == 0.0) d[i] = tiny;
                const double f = dl[i] / d[i];
                dl[i] = f;
                d[i + 1] -= f * du[i];
                du2[i] = 0.0;
                // right-hand side forward step (no swap)
                x[i + 1] -= f * x[i];
            } else {
                const double f = d[i] / dl[i];
                d[i] = dl[i];
                dl[i] = f;
                const double t = du[i];
                du[i] = d[i + 1];
                d[i + 1] = t - f * d[i + 1];
                if (i < k - 2) {
                    du2[i] = du[i + 1];
                    du[i + 1] = -f * du[i + 1];
                }
                const double xt = x[i];
                x[i] = x[i + 1];
                x[i + 1] = xt - f * x[i + 1];
            }
        }
        if (d[k - 1] == 0.0) d[k - 1] = tiny;
        // back substitution with the upper band (d, du, du2)
        x[k - 1] /= d[k - 1];
        if (k > 1) x[k - 2] = (x[k - 2] - du[k - 2] * x[k - 1]) / d[k - 2];
        for (int i = k - 3; i >= 0; --i) x[i] = (x[i] - du[i] * x[i + 1] - du2[i] * x[i + 2]) / d[i];
        sn = 0.0;
        for (int i = 0; i < k; ++i) sn += x[i] * x[i];
        sn = sqrt(sn);
        for (int i = 0; i < k; ++i) x[i] /= sn;
    }
    for (int i = 0; i < k; ++i) s_out[i] = make_double2(x[i], 0.0);
    st->theta = theta;
    result[0] = theta;
    result[1] = beta[k - 1] * fabs(x[k - 1]);
    result[3] = static_cast<double>(k);
}

// result[2] = sqrt(sum partials)
__global__ void k_resid_finalize(const double* __restrict__ partial, int nb, const LzState* __restrict__ st,
                                 double* __restrict__ result) {
    if (st->steps == 0) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partial[b];
    result[2] = sqrt(s);
}

struct LzLayout {
    size_t state, partial, coef, svec, work, omega, tmp, x32, y32, total;
};

LzLayout lz_layout(int64_t D, int32_t m, int32_t precision) {
    LzLayout L{};
    size_t off = 0;
    L.state = off;
    off = align_up(off + sizeof(LzState), 256);
    L.partial = off;
    off = align_up(off + sizeof(double2) * size_t(m + 1) * kMaxRedBlocks, 256);
    L.coef = off;
    off = align_up(off + sizeof(double2) * size_t(m + 1), 256);
    L.svec = off;
    off = align_up(off + sizeof(double2) * size_t(m + 1), 256);
    L.work = off;
    off = align_up(off + sizeof(double) * 5 * size_t(m + 1), 256);
    L.omega = off;
    off = align_up(off + sizeof(double) * 3 * size_t(m + 2), 256);
    L.tmp = off;
    off = align_up(off + sizeof(double2) * size_t(D), 256);
    L.x32 = L.y32 = off;
    if (precision == MRMF_PREC_C_IN_Z) {
        off = align_up(off + sizeof(float2) * size_t(D), 256);
        L.y32 = off;
        off = align_up(off + sizeof(float2) * size_t(D), 256);
    }
    L.total = off;
    return L;
}

int grid_for(int64_t n) {
    const int64_t b = (n + kRB - 1) / kRB;
    return static_cast<int>(b < 65536 ? (b < 1 ? 1 : b) : 65536);
}

}  // namespace
}  // namespace mrmf

using namespace mrmf;

extern "C" {

mrmf_status mrmf_reduce_scratch_bytes(int64_t n, size_t* bytes) {
    if (n < 0 || !bytes) return MRMF_E_INVALID_ARG;
    *bytes = align_up(sizeof(double2) * kMaxRedBlocks, 256);
    return MRMF_OK;
}

mrmf_status mrmf_dot_z(int64_t n, const void* d_a, const void* d_b, double* d_out, void* d_scratch,
                       size_t scratch_bytes, mrmf_stream stream) {
    if (n < 0 || !d_a || !d_b || !d_out || !d_scratch) return MRMF_E_INVALID_ARG;
    if (scratch_bytes < sizeof(double2) * kMaxRedBlocks) return MRMF_E_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int nb = red_blocks(n);
    auto* part = static_cast<double2*>(d_scratch);
    hipLaunchKernelGGL(k_dot_partial, dim3(nb), dim3(kRB), 0, s, n, static_cast<const double2*>(d_a),
                       static_cast<const double2*>(d_b), part, nullptr);
    hipLaunchKernelGGL(k_dot_finalize, dim3(1), dim3(1), 0, s, part, nb, d_out);
    return launch_status();
}

mrmf_status mrmf_norm_z(int64_t n, const void* d_a, double* d_out, void* d_scratch, size_t scratch_bytes,
                        mrmf_stream stream) {
    if (n < 0 || !d_a || !d_out || !d_scratch) return MRMF_E_INVALID_ARG;
    if (scratch_bytes < sizeof(double) * kMaxRedBlocks) return MRMF_E_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int nb = red_blocks(n);
    auto* part = static_cast<double*>(d_scratch);
    hipLaunchKernelGGL(k_norm2_partial, dim3(nb), dim3(kRB), 0, s, n, static_cast<const double2*>(d_a), part,
                       nullptr);
    hipLaunchKernelGGL(k_scalar_finalize, dim3(1), dim3(1), 0, s, part, nb, d_out, 1);
    return launch_status();
}

mrmf_status mrmf_lanczos_counts(const void* d_scratch, int32_t* d_out, mrmf_stream stream) {
    if (!d_scratch || !d_out || !aligned(d_scratch, 256) || !aligned(d_out, 4)) return MRMF_E_INVALID_ARG;
    // n_second and n_pro are adjacent in the state at the start of the scratch
    const unsigned char* st = static_cast<const unsigned char*>(d_scratch) + offsetof(LzState, n_second);
    static_assert(offsetof(LzState, n_pro) == offsetof(LzState, n_second) + sizeof(int32_t), "LzState layout");
    return hip_status(hipMemcpyAsync(d_out, st, 2 * sizeof(int32_t), hipMemcpyDeviceToDevice,
                                     static_cast<hipStream_t>(stream)));
}

mrmf_status mrmf_lanczos_scratch_bytes(mrmf_plan plan, int32_t m, int32_t precision, size_t* bytes) {
    if (!plan) return MRMF_E_INVALID_ARG;
    return lanczos_scratch_bytes(plan->D, m, precision, bytes);
}

}  // extern "C"

namespace mrmf {

mrmf_status lanczos_scratch_bytes(int64_t D, int32_t m, int32_t precision, size_t* bytes) {
    if (!bytes || m < 1 || m > 100000) return MRMF_E_INVALID_ARG;
    if (precision != MRMF_PREC_Z && precision != MRMF_PREC_C_IN_Z) return MRMF_E_INVALID_ARG;
    *bytes = lz_layout(D, m, precision).total;
    return MRMF_OK;
}

// The recurrence for any map of dimension D: mv_z applies it to a c128 vector, mv_c (C_IN_Z form) to a
// c64 one; both enqueue on the stream and honour the `stopped` flag.
mrmf_status lanczos_run(int64_t D, const MatvecOp& mv_z, const MatvecOp& mv_c, int32_t precision, int32_t m,
                        int32_t reorth, const void* d_v0, void* d_V, double* d_alpha, double* d_beta,
                        double* d_result, void* d_u, void* d_scratch, size_t scratch_bytes, mrmf_stream stream) {
    if (!d_v0 || !d_V || !d_alpha || !d_beta || !d_result || !d_u || !d_scratch) return MRMF_E_INVALID_ARG;
    if (m < 1 || m > 100000) return MRMF_E_INVALID_ARG;
    if (precision != MRMF_PREC_Z && precision != MRMF_PREC_C_IN_Z) return MRMF_E_INVALID_ARG;
    if (precision == MRMF_PREC_C_IN_Z && !mv_c) return MRMF_E_INVALID_ARG;
    if (reorth != MRMF_REORTH_CGS2 && reorth != MRMF_REORTH_NONE && reorth != MRMF_REORTH_CGS2_COND &&
        reorth != MRMF_REORTH_PARTIAL)
        return MRMF_E_INVALID_ARG;
    if (!aligned(d_scratch, 256) || !aligned(d_V, 16) || !aligned(d_u, 16) || !aligned(d_v0, 16))
        return MRMF_E_INVALID_ARG;
    const LzLayout Lo = lz_layout(D, m, precision);
    if (scratch_bytes < Lo.total) return MRMF_E_WORKSPACE;
    const size_t vb = sizeof(double2) * size_t(D);
    if (ranges_overlap(d_V, vb * size_t(m + 1), d_u, vb) || ranges_overlap(d_V, vb * size_t(m + 1), d_v0, vb))
        return MRMF_E_INVALID_ARG;

    hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned char* sc = static_cast<unsigned char*>(d_scratch);
    auto* st = reinterpret_cast<LzState*>(sc + Lo.state);
    const int32_t* stopped = &st->stopped;
    auto* part_d = reinterpret_cast<double*>(sc + Lo.partial);
    auto* part_z = reinterpret_cast<double2*>(sc + Lo.partial);
    auto* coef = reinterpret_cast<double2*>(sc + Lo.coef);
    auto* svec = reinterpret_cast<double2*>(sc + Lo.svec);
    auto* work = reinterpret_cast<double*>(sc + Lo.work);
    auto* omega = reinterpret_cast<double*>(sc + Lo.omega);
    auto* tmp = reinterpret_cast<double2*>(sc + Lo.tmp);
    auto* x32 = reinterpret_cast<float2*>(sc + Lo.x32);
    auto* y32 = reinterpret_cast<float2*>(sc + Lo.y32);
    auto* V = static_cast<double2*>(d_V);
    auto* u = static_cast<double2*>(d_u);
    const bool c32 = precision == MRMF_PREC_C_IN_Z;
    const int nb = red_blocks(D);
    const int g = grid_for(D);
    auto row = [&](int j) { return V + int64_t(j) * D; };

    // v_0 = v0 / ||v0||
    hipLaunchKernelGGL(k_norm2_partial, dim3(nb), dim3(kRB), 0, s, D, static_cast<const double2*>(d_v0), part_d,
                       nullptr);
    hipLaunchKernelGGL(k_init_finalize, dim3(1), dim3(1), 0, s, part_d, nb, st);
    hipLaunchKernelGGL(k_scale, dim3(g), dim3(kRB), 0, s, D, static_cast<const double2*>(d_v0), row(0), &st->nrm0,
                       c32 ? x32 : nullptr, stopped);
    mrmf_status rc = launch_status();
    if (rc != MRMF_OK) return rc;

    for (int j = 0; j < m; ++j) {
        double2* w = row(j + 1);
        // w = H v_j (the c64 form leaves H v_j in y32, read as it is by the next two kernels); alpha_j; then
        // the three-term update in one pass that also leaves the partial sums of ||w||^2 in part_d
        if (c32) {
            rc = mv_c(x32, y32, s, stopped);
            if (rc != MRMF_OK) return rc;
            hipLaunchKernelGGL(k_dot_partial32, dim3(nb), dim3(kRB), 0, s, D, row(j), y32, part_z, stopped);
        } else {
            rc = mv_z(row(j), w, s, stopped);
            if (rc != MRMF_OK) return rc;
            hipLaunchKernelGGL(k_dot_partial, dim3(nb), dim3(kRB), 0, s, D, row(j), w, part_z, stopped);
        }
        hipLaunchKernelGGL(k_alpha_finalize, dim3(1), dim3(1), 0, s, part_z, nb, d_alpha + j, stopped);
        hipLaunchKernelGGL(k_three_term_norm, dim3(nb), dim3(kRB), 0, s, D, w, c32 ? y32 : nullptr, row(j),
                           j > 0 ? row(j - 1) : nullptr, d_alpha + j, j > 0 ? d_beta + (j - 1) : nullptr, part_d,
                           stopped);
        if (reorth == MRMF_REORTH_CGS2 || reorth == MRMF_REORTH_CGS2_COND) {
            const int k = j + 1;
            const bool cond = reorth == MRMF_REORTH_CGS2_COND;
            if (cond) hipLaunchKernelGGL(k_cgs_norm, dim3(1), dim3(1), 0, s, part_d, nb, 1, st);
            for (int pass = 0; pass < 2; ++pass) {
                // the second pass of the conditional form runs (its kernels return at once otherwise)
                // only when the device-side test after the first pass asked for it
                const int32_t* stop = pass == 1 && cond ? &st->skip2 : stopped;
                if (pass == 1 && cond) {
                    hipLaunchKernelGGL(k_norm2_partial, dim3(nb), dim3(kRB), 0, s, D, w, part_d, stopped);
                    hipLaunchKernelGGL(k_cgs_norm, dim3(1), dim3(1), 0, s, part_d, nb, 0, st);
                }
                hipLaunchKernelGGL(k_gemvt_partial, dim3(nb, (k + kGroup - 1) / kGroup), dim3(kRB), 0, s, D, V, k,
                                   w, part_z, nb, stop);
                hipLaunchKernelGGL(k_gemvt_finalize, dim3((k + 63) / 64), dim3(64), 0, s, k, nb, part_z, coef,
                                   stop);
                hipLaunchKernelGGL(k_gemv_acc, dim3(g), dim3(kRB), 0, s, D, V, k, nullptr, coef, w, 0, -1.0, stop);
            }
            // ||w|| after the passes
            hipLaunchKernelGGL(k_norm2_partial, dim3(nb), dim3(kRB), 0, s, D, w, part_d, stopped);
        }
        if (reorth == MRMF_REORTH_PARTIAL) {
            // estimate the loss of orthogonality from ||w||; only when it calls for one, a Gram-Schmidt pass
            // against v_0 .. v_j and a new norm (the skipped kernels return at once, and the partial sums of
            // ||w||^2 from the three-term pass stay for k_beta_finalize)
            const int k = j + 1;
            const double eps = c32 ? 1.1920928955078125e-07 : 2.220446049250313e-16;  // 2^-23 or 2^-52
            hipLaunchKernelGGL(k_pro_estimate, dim3(1), dim3(kRB), 0, s, part_d, nb, j, m, D, eps, d_alpha,
                               d_beta, omega, st);
            const int32_t* stop = &st->skip_pro;
            hipLaunchKernelGGL(k_gemvt_partial, dim3(nb, (k + kGroup - 1) / kGroup), dim3(kRB), 0, s, D, V, k, w,
                               part_z, nb, stop);
            hipLaunchKernelGGL(k_gemvt_finalize, dim3((k + 63) / 64), dim3(64), 0, s, k, nb, part_z, coef, stop);
            hipLaunchKernelGGL(k_gemv_acc, dim3(g), dim3(kRB), 0, s, D, V, k, nullptr, coef, w, 0, -1.0, stop);
            hipLaunchKernelGGL(k_norm2_partial, dim3(nb), dim3(kRB), 0, s, D, w, part_d, stop);
        }
        hipLaunchKernelGGL(k_beta_finalize, dim3(1), dim3(1), 0, s, part_d, nb, j, j == m - 1 ? 1 : 0, d_alpha,
                           d_beta, st);
        if (j < m - 1)
            hipLaunchKernelGGL(k_scale, dim3(g), dim3(kRB), 0, s, D, w, w, d_beta + j, c32 ? x32 : nullptr,
                               stopped);
        rc = launch_status();
        if (rc != MRMF_OK) return rc;
    }
    // lowest Ritz pair of T, Ritz vector u = sum_i s_i v_i, explicit residual with the FP64 map
    hipLaunchKernelGGL(k_tridiag_lowest, dim3(1), dim3(1), 0, s, d_alpha, d_beta, m, st, work, svec, d_result);
    hipLaunchKernelGGL(k_gemv_acc, dim3(g), dim3(kRB), 0, s, D, V, m, &st->steps, svec, u, 1, 1.0, nullptr);
    hipLaunchKernelGGL(k_norm2_partial, dim3(nb), dim3(kRB), 0, s, D, u, part_d, nullptr);
    hipLaunchKernelGGL(k_unorm_finalize, dim3(1), dim3(1), 0, s, part_d, nb, st);
    hipLaunchKernelGGL(k_scale, dim3(g), dim3(kRB), 0, s, D, u, u, &st->unrm, nullptr, &st->skip_u);
    rc = launch_status();
    if (rc != MRMF_OK) return rc;
    rc = mv_z(u, tmp, s, nullptr);
    if (rc != MRMF_OK) return rc;
    hipLaunchKernelGGL(k_resid_partial, dim3(nb), dim3(kRB), 0, s, D, tmp, u, st, part_d);
    hipLaunchKernelGGL(k_resid_finalize, dim3(1), dim3(1), 0, s, part_d, nb, st, d_result);
    return launch_status();
}

}  // namespace mrmf

extern "C" {

mrmf_status mrmf_lanczos(mrmf_plan plan, const void* d_ws, const double* d_theta_z, const float* d_theta_c,
                         int32_t precision, int32_t m, int32_t reorth, const void* d_v0, void* d_V,
                         double* d_alpha, double* d_beta, double* d_result, void* d_u, void* d_scratch,
                         size_t scratch_bytes, mrmf_stream stream) {
    if (!plan || !d_ws || !d_theta_z) return MRMF_E_INVALID_ARG;
    if (precision == MRMF_PREC_C_IN_Z && !d_theta_c) return MRMF_E_INVALID_ARG;
    // the recurrence keeps Re<v|Hv> only and its Ritz values are eigenvalues of H only for Hermitian H
    if (!plan->hermitian) return MRMF_E_NOT_HERMITIAN;
    const MatvecOp mv_z = [&](const void* x, void* y, hipStream_t s, const int32_t* stop) {
        return matvec_z_impl(plan, d_ws, d_theta_z, x, y, s, stop);
    };
    const MatvecOp mv_c = [&](const void* x, void* y, hipStream_t s, const int32_t* stop) {
        return matvec_c_impl(plan, d_ws, d_theta_c, x, y, s, stop);
    };
    return lanczos_run(plan->D, mv_z, mv_c, precision, m, reorth, d_v0, d_V, d_alpha, d_beta, d_result, d_u,
                       d_scratch, scratch_bytes, stream);
}

}  // extern "C"
