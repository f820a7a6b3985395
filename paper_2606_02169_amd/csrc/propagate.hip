// Time propagation x(t) = exp(-i H t) x0 through the matrix-free map (the exact flat-basis propagation
// under rebuilt or driven couplings named as a use case in Sec. VII and Sec. VIII).
//
// Each step of length dt applies the Chebyshev expansion of the exponential (Jacobi-Anger):
//     exp(-i H dt) = exp(-i b dt) sum_k (2 - delta_k0) (-i)^k J_k(a dt) T_k(Ht),   Ht = (H - b) / a,
// where [b - a, b + a] contains the spectrum of H (caller's bounds; mrmf_plan_norm_bound gives a safe
// symmetric one).  T_k(Ht) v follows the three-term recurrence phi_k = 2 Ht phi_{k-1} - phi_{k-2}: one
// launch of the plan's specialized kernel with a Chebyshev-step epilogue per term (it reads the row's
// phi_{k-2} and accumulator and writes phi_k and the accumulator, so H phi never goes to memory), or, for
// plans on the generic kernel, a matvec and a fused vector update; the series is cut where the remaining
// Bessel weights sum below the tolerance (|T_k(Ht)| <= 1 on the spectrum).  A piecewise-constant drive supplies one
// parameter vector per step (theta + s * theta_stride): the plan and its kernels are reused as they are.
// With a fixed H, q consecutive steps are one step of length q dt (the exponential of a fixed H composes:
// exp(-i H dt)^q = exp(-i H q dt)), whose series needs about a q |dt| + O((a q |dt|)^(1/3)) terms instead
// of q times those of one step, and is truncated once instead of q times.
#include <algorithm>
#include <climits>
#include <cmath>
#include <vector>

#include "mrmf_internal.h"

namespace mrmf {
namespace {

constexpr int kPB = 256;

int prop_grid(int64_t n) {
    const int64_t b = (n + kPB - 1) / kPB;
    return static_cast<int>(b < 16384 ? (b < 1 ? 1 : b) : 16384);
}

// acc = c0 * state, cur = state, prev = 0 (state may be acc itself: each element is read before it is
// written; prev starts at zero because the fused first step reads it with weight 0)
__global__ __launch_bounds__(kPB) void k_cheb_init(int64_t n, const double2* state, double2* cur, double2* prev,
                                                   double2* acc, double c0r, double c0i) {
    for (int64_t i = int64_t(blockIdx.x) * kPB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kPB) {
        const double2 v = state[i];
        cur[i] = v;
        prev[i] = make_double2(0.0, 0.0);
        acc[i] = make_double2(c0r * v.x - c0i * v.y, c0r * v.y + c0i * v.x);
    }
}

// phi_new = alpha hv + beta cur + gamma prev (prev not read when null); prev = phi_new; acc += c phi_new
__global__ __launch_bounds__(kPB) void k_cheb_update(int64_t n, const double2* __restrict__ hv,
                                                     const double2* __restrict__ cur, double2* __restrict__ prev,
                                                     double2* __restrict__ acc, double alpha, double beta,
                                                     double gamma, int use_prev, double cr, double ci) {
    for (int64_t i = int64_t(blockIdx.x) * kPB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kPB) {
        const double2 h = hv[i], u = cur[i];
        double2 p = make_double2(alpha * h.x + beta * u.x, alpha * h.y + beta * u.y);
        if (use_prev) {
            const double2 q = prev[i];
            p.x += gamma * q.x;
            p.y += gamma * q.y;
        }
        prev[i] = p;
        double2 a = acc[i];
        a.x += cr * p.x - ci * p.y;
        a.y += cr * p.y + ci * p.x;
        acc[i] = a;
    }
}

// Operator norm of a one-site factor: at most one nonzero per row and column, so the largest entry.
double local_norm(const mrmf_plan_t* p, int site, int op) {
    double m = 0.0;
    for (int n = 0; n < p->d[site]; ++n) m = std::fmax(m, std::fabs(local_factor_host(p, site, op, n)));
    return m;
}

}  // namespace

// J_0(z) .. J_{K}(z) for z >= 0 by Miller's backward recurrence J_{k-1} = (2k / z) J_k - J_{k+1}, started
// far above z with an arbitrary small seed and normalised by J_0 + 2 sum_k J_{2k} = 1; K is the smallest
// index with 2 sum_{k > K} |J_k| <= tol.  Returns K + 1, or 0 when more than cap terms would be needed.
int cheb_bessel(double z, double tol, int cap, std::vector<double>& J) {
    J.clear();
    if (z < 1e-300) {
        J.push_back(1.0);
        return 1;
    }
    const double top = z + 60.0 + 20.0 * std::cbrt(z);
    if (top > 4.0 * double(cap) + 64.0) return 0;
    int kst = static_cast<int>(top);
    kst += kst & 1;
    std::vector<double> j(kst + 2, 0.0);
    j[kst] = 1e-280;
    for (int k = kst; k >= 1; --k) {
        j[k - 1] = (2.0 * k / z) * j[k] - j[k + 1];
        if (std::fabs(j[k - 1]) > 1e250)
            for (int i = k - 1; i <= kst; ++i) j[i] *= 1e-250;
    }
    double s = j[0];
    for (int k = 2; k <= kst; k += 2) s += 2.0 * j[k];
    for (int k = 0; k <= kst; ++k) j[k] /= s;
    double tail = 0.0;
    int K = kst;
    for (int k = kst; k >= 1; --k) {
        if (tail + 2.0 * std::fabs(j[k]) > tol) break;
        tail += 2.0 * std::fabs(j[k]);
        K = k - 1;
    }
    if (K + 1 > cap) return 0;
    J.assign(j.begin(), j.begin() + K + 1);
    return K + 1;
}

size_t propagate_scratch_bytes(int64_t n) { return 3 * (size_t(n) * 16 + 256); }

mrmf_status propagate_run(int64_t n, int32_t n_params, const ThetaMatvecOp& mv, const ChebStepOp* step,
                          const std::function<bool()>& fused_ready, bool merge, const double* d_theta,
                          int64_t theta_stride, double dt, int32_t n_steps, double e_min, double e_max, double tol,
                          const void* d_x0, void* d_x, void* d_scratch, size_t scratch_bytes, int32_t* h_n_terms,
                          hipStream_t s) {
    if (!d_x0 || !d_x || !d_scratch) return MRMF_E_INVALID_ARG;
    if (n_steps < 0 || theta_stride < 0 || !std::isfinite(dt) || !std::isfinite(e_min) || !std::isfinite(e_max) ||
        !(e_max > e_min) || !(tol > 0.0) || !(tol < 1.0))
        return MRMF_E_INVALID_ARG;
    if (!aligned(d_x0, 16) || !aligned(d_x, 16) || !aligned(d_scratch, 256)) return MRMF_E_INVALID_ARG;
    const size_t vb = size_t(n) * 16;
    const size_t need = propagate_scratch_bytes(n);
    if (scratch_bytes < need) return MRMF_E_WORKSPACE;
    if ((d_x0 != d_x && ranges_overlap(d_x0, vb, d_x, vb)) || ranges_overlap(d_scratch, need, d_x, vb) ||
        ranges_overlap(d_scratch, need, d_x0, vb))
        return MRMF_E_INVALID_ARG;
    const double a = 0.5 * (e_max - e_min), b = 0.5 * (e_max + e_min);
    // the coefficients c_k = (2 - delta_k0) (-i)^k J_k(a h) exp(-i b h) of a step of length h (J_k(-z) =
    // (-1)^k J_k(z) for h < 0); 0 terms when the series needs more than cap
    auto coefficients = [&](double h, int cap, std::vector<double>& cr, std::vector<double>& ci) {
        std::vector<double> J;
        const int nt = cheb_bessel(a * std::fabs(h), tol, cap, J);
        cr.assign(nt, 0.0);
        ci.assign(nt, 0.0);
        const double pr = std::cos(b * h), pi = -std::sin(b * h);
        for (int k = 0; k < nt; ++k) {
            double w = (k == 0 ? 1.0 : 2.0) * J[k];
            if (h < 0 && (k & 1)) w = -w;
            double ur = 0.0, ui = 0.0;  // (-i)^k
            switch (k & 3) {
                case 0: ur = 1.0; break;
                case 1: ui = -1.0; break;
                case 2: ur = -1.0; break;
                default: ui = 1.0; break;
            }
            cr[k] = w * (ur * pr - ui * pi);
            ci[k] = w * (ur * pi + ui * pr);
        }
        return nt;
    };
    // steps per series: 1, or for a fixed H (merge) the largest q <= n_steps whose step q dt keeps the
    // series within kMergeTerms terms (exp(-i H dt)^q = exp(-i H q dt); one truncation instead of q, and
    // the terms grow about like a q |dt| rather than q times)
    constexpr int kMergeTerms = 2048;
    std::vector<double> cr, ci;
    const int nt1 = coefficients(dt, 1 << 20, cr, ci);
    if (nt1 == 0) return MRMF_E_UNSUPPORTED;
    int q = 1;
    if (theta_stride == 0 && merge && n_steps > 1) {
        std::vector<double> tr, ti;
        for (q = n_steps; q > 1; q = (q + 1) / 2)
            if (coefficients(q * dt, kMergeTerms, tr, ti) > 0) break;
    }
    char* base = static_cast<char*>(d_scratch);
    const size_t slot = vb + 256 - (vb % 256 ? vb % 256 : 256);  // 256-B aligned slots
    double2* v0 = reinterpret_cast<double2*>(base);
    double2* v1 = reinterpret_cast<double2*>(base + slot);
    double2* hv = reinterpret_cast<double2*>(base + 2 * slot);
    double2* x = static_cast<double2*>(d_x);
    const int grid = prop_grid(n);
    const bool fused = step != nullptr && n_steps > 0 && nt1 > 1 && fused_ready();
    int64_t total = 0;
    int qcur = 0;  // steps of the series whose coefficients cr, ci hold
    for (int st = 0; st < n_steps;) {
        const int qs = std::min(q, n_steps - st);  // this series covers steps st .. st + qs - 1
        if (qs != qcur) {
            const int nt = coefficients(qs * dt, qs == 1 ? 1 << 20 : kMergeTerms, cr, ci);
            if (nt == 0) return MRMF_E_UNSUPPORTED;
            qcur = qs;
        }
        const int nt = static_cast<int>(cr.size());
        total += nt;
        const double* th = n_params > 0 ? d_theta + int64_t(st) * theta_stride : nullptr;
        const double2* state = st == 0 ? static_cast<const double2*>(d_x0) : x;
        double2* cur = v0;
        double2* prev = v1;
        hipLaunchKernelGGL(k_cheb_init, dim3(grid), dim3(kPB), 0, s, n, state, cur, prev, x, cr[0], ci[0]);
        mrmf_status rc = launch_status();
        if (rc != MRMF_OK) return rc;
        for (int k = 1; k < nt; ++k) {
            const bool first = k == 1;
            const double ea = (first ? 1.0 : 2.0) / a, eb = -(first ? 1.0 : 2.0) * b / a, eg = first ? 0.0 : -1.0;
            if (fused) {
                rc = (*step)(th, cur, prev, x, ea, eb, eg, cr[k], ci[k], s);
                if (rc != MRMF_OK) return rc;
            } else {
                rc = mv(th, cur, hv, s);
                if (rc != MRMF_OK) return rc;
                hipLaunchKernelGGL(k_cheb_update, dim3(grid), dim3(kPB), 0, s, n, hv, cur, prev, x, ea, eb, eg,
                                   first ? 0 : 1, cr[k], ci[k]);
                rc = launch_status();
                if (rc != MRMF_OK) return rc;
            }
            double2* t = cur;
            cur = prev;
            prev = t;
        }
        st += qs;
    }
    if (h_n_terms) *h_n_terms = n_steps == 0 ? nt1 : static_cast<int32_t>(std::min<int64_t>(total, INT32_MAX));
    if (n_steps == 0 && d_x0 != d_x) return hip_status(hipMemcpyAsync(d_x, d_x0, vb, hipMemcpyDeviceToDevice, s));
    return MRMF_OK;
}

}  // namespace mrmf

using namespace mrmf;

extern "C" {

mrmf_status mrmf_plan_norm_bound(mrmf_plan plan, const double* h_theta, double* bound) {
    if (!plan || !bound || (plan->n_params > 0 && !h_theta)) return MRMF_E_INVALID_ARG;
    double b = 0.0;
    for (const auto& t : plan->terms) {
        const double th = h_theta[t.param];
        if (!std::isfinite(th)) return MRMF_E_INVALID_ARG;
        double nrm = std::fabs(th) * std::hypot(t.w_re, t.w_im) * local_norm(plan, t.site_a, t.op_a);
        if (t.site_b >= 0) nrm *= local_norm(plan, t.site_b, t.op_b);
        b += nrm;
    }
    *bound = b;
    return MRMF_OK;
}

mrmf_status mrmf_cheb_bessel(double z, double tol, int32_t cap, double* h_out, int32_t* n_terms) {
    if (!n_terms || !(z >= 0.0) || !std::isfinite(z) || !(tol > 0.0) || !(tol < 1.0) || cap < 1)
        return MRMF_E_INVALID_ARG;
    std::vector<double> J;
    const int n = cheb_bessel(z, tol, cap, J);
    if (n == 0) return MRMF_E_UNSUPPORTED;
    if (h_out)
        for (int k = 0; k < n; ++k) h_out[k] = J[k];
    *n_terms = n;
    return MRMF_OK;
}

mrmf_status mrmf_propagate_scratch_bytes(mrmf_plan plan, size_t* bytes) {
    if (!plan || !bytes) return MRMF_E_INVALID_ARG;
    *bytes = propagate_scratch_bytes(plan->D);
    return MRMF_OK;
}

mrmf_status mrmf_propagate_z(mrmf_plan plan, const void* d_ws, const double* d_theta, int64_t theta_stride,
                             double dt, int32_t n_steps, double e_min, double e_max, double tol, const void* d_x0,
                             void* d_x, void* d_scratch, size_t scratch_bytes, int32_t* h_n_terms,
                             mrmf_stream stream) {
    if (!plan || !d_ws || (plan->n_params > 0 && !d_theta)) return MRMF_E_INVALID_ARG;
    if (!plan->hermitian) return MRMF_E_NOT_HERMITIAN;
    if (!aligned(d_ws, 256)) return MRMF_E_INVALID_ARG;
    const ThetaMatvecOp mv = [&](const double* th, const void* x, void* y, hipStream_t s) {
        return matvec_z_impl(plan, d_ws, th, x, y, s, nullptr);
    };
    // the specialized kernel with the Chebyshev-step epilogue does matvec and update in one pass (no
    // H phi vector written and read back); plans without a specialized kernel take the two-pass form
    const ChebStepOp step = [&](const double* th, const void* cur, void* prev, void* acc, double ea, double eb,
                                double eg, double cr, double ci, hipStream_t s) {
        return spec_launch_cheb(plan, th, cur, prev, acc, ea, eb, eg, cr, ci, s);
    };
    const auto fused_ready = [&]() {
        return plan->cfg[MRMF_DTYPE_Z].mode != MRMF_KERNEL_GENERIC && plan->cfg[MRMF_DTYPE_Z].cheb_fused != 0 &&
               spec_prepare(plan, kSlotCheb) == MRMF_OK;
    };
    return propagate_run(plan->D, plan->n_params, mv, &step, fused_ready, plan->cfg[MRMF_DTYPE_Z].cheb_merge != 0,
                         d_theta, theta_stride, dt, n_steps, e_min, e_max, tol, d_x0, d_x, d_scratch, scratch_bytes,
                         h_n_terms, static_cast<hipStream_t>(stream));
}

}  // extern "C"
