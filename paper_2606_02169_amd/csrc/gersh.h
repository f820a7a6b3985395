// Gershgorin ends of H(theta_s) for several coupling vectors theta_0 .. theta_{S-1} in one pass over the
// rows (device code shared by the full-basis and the sector bounds).
//
// H(theta) = sum_p theta_p h_p, every diagonal term and every channel carrying one coupling, so a row's
// diagonal entry is sum_p theta_p A_p and the channel sum of its radius is sum_p |theta_p| B_p, with
// A_p = sum of w_r f_a f_b over the diagonal terms of coupling p and B_p = sum of |w f_a f_b| over its
// channels whose source digits are in range.  A block tabulates every term's contribution over its digits
// in LDS (no coupling in it), a row sums its terms into A_p and B_p, and then every theta_s costs 2 P
// multiply-adds.  The ends are those of S separate one-vector passes up to the order of the sums.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "mrmf_internal.h"

namespace mrmf {

constexpr int kLinMaxParams = 8;     // couplings held in registers per row
constexpr int kLinTab = 2048;        // table entries of all terms together
constexpr int kLinMaxTerms = 256;
constexpr int kLinBlock = 256;

// Whether a plan or sector with these terms takes the one-pass form.
inline bool gersh_lin_fits(int n_params, const std::vector<int32_t>& d, const std::vector<DevDiag>& diags,
                           const std::vector<DevChan>& chans) {
    if (n_params > kLinMaxParams || diags.size() + chans.size() > size_t(kLinMaxTerms)) return false;
    int64_t entries = 0;
    for (const auto& g : diags) entries += int64_t(d[g.a]) * (g.b >= 0 ? d[g.b] : 1);
    for (const auto& c : chans) entries += int64_t(d[c.a]) * (c.b >= 0 ? d[c.b] : 1);
    return entries <= kLinTab;
}

struct GershLinLds {
    double tab[kLinTab];
    int4 td[kLinMaxTerms];  // per term: site a, site b (-1: none), d_b (1 without b), table offset
    int tq[kLinMaxTerms];   // per term: 2 p + (1 for a channel)
};

// The block's tables.  fac(op, tab, n): the local matrix element <n|O|n - q> at target digit n.
template <typename Fac>
__device__ void gersh_lin_tables(const PlanArgs& p, Fac fac, GershLinLds& L) {
    const int tid = threadIdx.x, nt = p.n_diag + p.n_chan;
    if (tid == 0) {
        int off = 0;
        for (int k = 0; k < nt; ++k) {
            const bool dg = k < p.n_diag;
            const int ta = dg ? p.diag[k].a : p.chan[k - p.n_diag].a;
            const int tb = dg ? p.diag[k].b : p.chan[k - p.n_diag].b;
            const int db = tb >= 0 ? p.site[tb].d : 1;
            L.td[k] = make_int4(ta, tb, db, off);
            L.tq[k] = 2 * (dg ? p.diag[k].param : p.chan[k - p.n_diag].param) + (dg ? 0 : 1);
            off += p.site[ta].d * db;
        }
    }
    __syncthreads();
    for (int k = 0; k < nt; ++k) {
        const int4 t = L.td[k];
        const int n = p.site[t.x].d * t.z;
        for (int e = tid; e < n; e += kLinBlock) {
            const int na = e / t.z, nb = e - na * t.z;
            double v;
            if (k < p.n_diag) {
                const DevDiag g = p.diag[k];
                double f = fac(g.opa, p.site[g.a].tab, na);
                if (g.b >= 0) f *= fac(g.opb, p.site[g.b].tab, nb);
                v = g.wr * f;
            } else {
                const DevChan ch = p.chan[k - p.n_diag];
                bool ok = na - ch.qa >= 0 && na - ch.qa < p.site[ch.a].d;
                double f = fac(ch.opa, p.site[ch.a].tab, na);
                if (ch.b >= 0) {
                    ok = ok && nb - ch.qb >= 0 && nb - ch.qb < p.site[ch.b].d;
                    f *= fac(ch.opb, p.site[ch.b].tab, nb);
                }
                v = ok ? fabs(f) * sqrt(ch.wr * ch.wr + ch.wi * ch.wi) : 0.0;
            }
            L.tab[t.w + e] = v;
        }
    }
    __syncthreads();
}

// One row (its digits in dig[site][threadIdx.x]): A_p and B_p, then the ends over the S vectors
// theta + s * stride folded into lo / hi.
__device__ __forceinline__ void gersh_lin_row(const PlanArgs& p, const GershLinLds& L,
                                              const uint8_t (*dig)[kLinBlock], const double* __restrict__ theta,
                                              int64_t stride, int32_t count, double& lo, double& hi) {
    const int tid = threadIdx.x, nt = p.n_diag + p.n_chan;
    double a[kLinMaxParams], b[kLinMaxParams];
#pragma unroll
    for (int q = 0; q < kLinMaxParams; ++q) a[q] = b[q] = 0.0;
    for (int k = 0; k < nt; ++k) {
        const int4 t = L.td[k];
        const int e = dig[t.x][tid] * t.z + (t.y >= 0 ? dig[t.y][tid] : 0);
        const double v = L.tab[t.w + e];
        const int tq = __builtin_amdgcn_readfirstlane(L.tq[k]);  // block-uniform
        const int q = tq >> 1;
#pragma unroll
        for (int u = 0; u < kLinMaxParams; ++u)
            if (u == q) {
                if (tq & 1) b[u] += v;
                else a[u] += v;
            }
    }
    for (int32_t s = 0; s < count; ++s) {
        const double* th = theta + s * stride;
        double dg = 0.0, rad = 0.0;
#pragma unroll
        for (int u = 0; u < kLinMaxParams; ++u)
            if (u < p.n_params) {
                dg += th[u] * a[u];
                rad += fabs(th[u]) * b[u];
            }
        lo = fmin(lo, dg - rad);
        hi = fmax(hi, dg + rad);
    }
}

// Block min / max of lo and hi to partial[2 blockIdx.x], partial[2 blockIdx.x + 1].
__device__ __forceinline__ void gersh_block_ends(double lo, double hi, double* slo, double* shi,
                                                 double* __restrict__ partial) {
    const int tid = threadIdx.x;
    slo[tid] = lo;
    shi[tid] = hi;
    __syncthreads();
    if (tid == 0) {
        for (int k = 1; k < kLinBlock; ++k) {
            lo = fmin(lo, slo[k]);
            hi = fmax(hi, shi[k]);
        }
        partial[2 * blockIdx.x] = lo;
        partial[2 * blockIdx.x + 1] = hi;
    }
}

// One block of kLinBlock threads: the minimum of partial[2 b] and the maximum of partial[2 b + 1] over the nb
// blocks of a bounds pass to out[0], out[1] (min and max: the same result in any order).
__device__ __forceinline__ void gersh_finalize_block(const double* __restrict__ partial, int nb,
                                                     double* __restrict__ out) {
    __shared__ double slo[kLinBlock], shi[kLinBlock];
    const int tid = threadIdx.x;
    double lo = __builtin_inf(), hi = -__builtin_inf();
    for (int b = tid; b < nb; b += kLinBlock) {
        lo = fmin(lo, partial[2 * b]);
        hi = fmax(hi, partial[2 * b + 1]);
    }
    slo[tid] = lo;
    shi[tid] = hi;
    __syncthreads();
    for (int w = kLinBlock / 2; w > 0; w >>= 1) {
        if (tid < w) {
            slo[tid] = fmin(slo[tid], slo[tid + w]);
            shi[tid] = fmax(shi[tid], shi[tid + w]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        out[0] = slo[0];
        out[1] = shi[0];
    }
}

}  // namespace mrmf
