// Restricted basis of a globally constrained sector (Sec. VI, case 2): every product state whose local
// digits sum to Q (fixed total magnetization for spins, fixed excitation number with bosons), stored
// packed in ascending full-basis order.  The lookup is a combinatorial ranking (the Lehmer-code-style
// option of Sec. VI.B) instead of a search or a hash: with C_k(q) the number of digit tuples of sites
// k..N-1 summing to q and R_k(q, v) = sum_{v' < v} C_{k+1}(q - v'),
//     rank(n_0 .. n_{N-1}) = sum_k R_k(Q_k, n_k),     Q_0 = Q,  Q_{k+1} = Q_k - n_k,
// and unranking walks the same tables site by site.  The source of a channel on sites i < j differs from
// the target only in n_i, n_j and in the remaining sums Q_k for i < k <= j, so its rank is the target's
// plus the change of those j - i + 1 table terms: no search and no table of labels to search.  The
// generic kernels here unrank each target row; the kernel generated for the sector (jit.cpp) reads the
// target's digits from a word per state that k_sector_pack writes into the workspace at upload.  A
// channel that changes the digit sum has no source in the sector (the failed membership test of
// Sec. VI.B) and is dropped when the sector is built; one-site ladder channels are such channels.
#include <algorithm>
#include <cstring>
#include <type_traits>
#include <vector>

#include "gersh.h"
#include "mrmf_internal.h"

namespace mrmf {
namespace {

constexpr int kSB = 256;

struct SectorArgs {
    PlanArgs p;              // chan: the sector's channels
    const int64_t* rt;       // rank tables: site k at rt + rto[k], entry (q, v) at q * (d_k + 1) + v
    const int64_t* rto;      // per-site offsets into rt
    int64_t Dr;
    int32_t Q, n_rt;         // digit sum, number of rank-table entries
};

SectorArgs sector_args(const mrmf_sector_t* S, const void* d_ws) {
    const unsigned char* b = static_cast<const unsigned char*>(d_ws);
    SectorArgs a;
    a.p.site = reinterpret_cast<const DevSite*>(b + S->off_site);
    a.p.chan = reinterpret_cast<const DevChan*>(b + S->off_chan);
    a.p.diag = reinterpret_cast<const DevDiag*>(b + S->off_diag);
    a.p.val = reinterpret_cast<const double*>(b + S->off_val);
    a.p.up = reinterpret_cast<const double*>(b + S->off_up);
    a.p.lofs = reinterpret_cast<const int32_t*>(b + S->off_lofs);
    a.p.D = S->Dr;
    a.p.N = S->N;
    a.p.n_chan = static_cast<int32_t>(S->chans.size());
    a.p.n_diag = static_cast<int32_t>(S->diags.size());
    a.p.n_params = S->n_params;
    a.rt = reinterpret_cast<const int64_t*>(b + S->off_rt);
    a.rto = reinterpret_cast<const int64_t*>(b + S->off_rto);
    a.Dr = S->Dr;
    a.Q = S->Q;
    a.n_rt = S->n_rt;
    return a;
}

// <n|O|n - q> of a local operator at target digit n (admissible n assumed)
template <typename R>
__device__ __forceinline__ R sfactor(const PlanArgs& p, int op, int tab, int n) {
    switch (op) {
        case MRMF_OP_Z: return static_cast<R>(p.val[tab + n]);
        case MRMF_OP_Z2: return static_cast<R>(p.val[tab + n] * p.val[tab + n]);
        case MRMF_OP_RAISE: return static_cast<R>(p.up[tab + n]);
        case MRMF_OP_LOWER: return static_cast<R>(p.up[tab + n + 1]);
        case MRMF_OP_RAISE2: return static_cast<R>(p.up[tab + n] * p.up[tab + n - 1]);
        case MRMF_OP_LOWER2: return static_cast<R>(p.up[tab + n + 1] * p.up[tab + n + 2]);
        default: return static_cast<R>(p.up[p.lofs[op - MRMF_OP_LOCAL_BASE] + n]);  // general one-site operator
    }
}

__device__ __forceinline__ int64_t rtab(const SectorArgs& a, int k, int q, int v) {
    return a.rt[a.rto[k] + int64_t(q) * (a.p.site[k].d + 1) + v];
}

// Digits and remaining sums of packed row r (rem[k] = Q_k).
__device__ __forceinline__ void unrank(const SectorArgs& a, int64_t r, uint8_t (*dig)[kSB], uint16_t (*rem)[kSB],
                                       int tid) {
    int q = a.Q;
    int64_t left = r;
    for (int k = 0; k < a.p.N; ++k) {
        const int d = a.p.site[k].d;
        const int vmax = q < d - 1 ? q : d - 1;
        const int64_t* R = a.rt + a.rto[k] + int64_t(q) * (d + 1);
        int v = 0;
        while (v < vmax && R[v + 1] <= left) ++v;
        dig[k][tid] = static_cast<uint8_t>(v);
        rem[k][tid] = static_cast<uint16_t>(q);
        left -= R[v];
        q -= v;
    }
}

template <typename R>
__global__ __launch_bounds__(kSB) void k_sector_matvec(SectorArgs a, const R* __restrict__ theta,
                                                       const typename Cx<R>::T* __restrict__ x,
                                                       typename Cx<R>::T* __restrict__ y,
                                                       const int32_t* __restrict__ skip) {
    using C = typename Cx<R>::T;
    if (skip != nullptr && *skip != 0) return;
    __shared__ uint8_t dig[kMaxSites][kSB];
    __shared__ uint16_t rem[kMaxSites][kSB];
    const int tid = threadIdx.x;
    const PlanArgs& p = a.p;
    for (int64_t r = int64_t(blockIdx.x) * kSB + tid; r < a.Dr; r += int64_t(gridDim.x) * kSB) {
        unrank(a, r, dig, rem, tid);
        R dr = 0, di = 0;
        for (int k = 0; k < p.n_diag; ++k) {
            const DevDiag g = p.diag[k];
            R f = sfactor<R>(p, g.opa, p.site[g.a].tab, dig[g.a][tid]);
            if (g.b >= 0) f *= sfactor<R>(p, g.opb, p.site[g.b].tab, dig[g.b][tid]);
            const R th = theta[g.param];
            dr += th * static_cast<R>(g.wr) * f;
            di += th * static_cast<R>(g.wi) * f;
        }
        const C xf = x[r];
        R ar = dr * xf.x - di * xf.y;
        R ai = dr * xf.y + di * xf.x;
        for (int c = 0; c < p.n_chan; ++c) {
            const DevChan ch = p.chan[c];
            const int na = dig[ch.a][tid], nb = dig[ch.b][tid];
            const int sa = na - ch.qa, sb = nb - ch.qb;
            if (sa < 0 || sa >= p.site[ch.a].d || sb < 0 || sb >= p.site[ch.b].d) continue;
            // source rank: the terms of sites i..j change (i < j the two sites)
            const bool a_first = ch.a < ch.b;
            const int i = a_first ? ch.a : ch.b, j = a_first ? ch.b : ch.a;
            const int ni = a_first ? na : nb, nsi = a_first ? sa : sb;
            const int nj = a_first ? nb : na, nsj = a_first ? sb : sa;
            const int dq = nsi - ni;  // the remaining sums after site i drop by dq
            const int qi = rem[i][tid];
            int64_t drank = rtab(a, i, qi, nsi) - rtab(a, i, qi, ni);
            for (int k = i + 1; k < j; ++k) {
                const int qk = rem[k][tid], nk = dig[k][tid];
                drank += rtab(a, k, qk - dq, nk) - rtab(a, k, qk, nk);
            }
            const int qj = rem[j][tid];
            drank += rtab(a, j, qj - dq, nsj) - rtab(a, j, qj, nj);
            const R f = sfactor<R>(p, ch.opa, p.site[ch.a].tab, na) * sfactor<R>(p, ch.opb, p.site[ch.b].tab, nb);
            const R th = theta[ch.param] * f;
            const R cr = th * static_cast<R>(ch.wr), ci = th * static_cast<R>(ch.wi);
            const C xs = x[r + drank];
            ar += cr * xs.x - ci * xs.y;
            ai += cr * xs.y + ci * xs.x;
        }
        C out;
        out.x = ar;
        out.y = ai;
        y[r] = out;
    }
}

// The same map with the rank tables, their per-site offsets and the digits / remaining sums of the
// block's rows in LDS (dynamic shared memory sized for this lattice): unranking and the source-rank
// updates then read LDS only.  RT is int32_t when every rank fits, else int64_t.
template <typename R, typename RT>
__global__ __launch_bounds__(kSB) void k_sector_matvec_lds(SectorArgs a, const R* __restrict__ theta,
                                                           const typename Cx<R>::T* __restrict__ x,
                                                           typename Cx<R>::T* __restrict__ y,
                                                           const int32_t* __restrict__ skip) {
    using C = typename Cx<R>::T;
    if (skip != nullptr && *skip != 0) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = a.p.N;
    RT* lrt = reinterpret_cast<RT*>(smem);
    int32_t* lro = reinterpret_cast<int32_t*>(smem + sizeof(RT) * size_t(a.n_rt));  // offset of site k
    int32_t* ld1 = lro + N;                                                         // d_k + 1
    uint16_t* rem = reinterpret_cast<uint16_t*>(ld1 + N);                            // [N][kSB]
    uint8_t* dig = reinterpret_cast<uint8_t*>(rem + size_t(N) * kSB);                // [N][kSB]
    const int tid = threadIdx.x;
    for (int i = tid; i < a.n_rt; i += kSB) lrt[i] = static_cast<RT>(a.rt[i]);
    for (int k = tid; k < N; k += kSB) {
        lro[k] = static_cast<int32_t>(a.rto[k]);
        ld1[k] = a.p.site[k].d + 1;
    }
    __syncthreads();
    const PlanArgs& p = a.p;
    auto rt = [&](int k, int q, int v) -> int64_t { return lrt[lro[k] + q * ld1[k] + v]; };
    for (int64_t r = int64_t(blockIdx.x) * kSB + tid; r < a.Dr; r += int64_t(gridDim.x) * kSB) {
        {   // unrank: the digit of site k is the v with R_k(q, v) <= left < R_k(q, v + 1)
            int q = a.Q;
            int64_t left = r;
            for (int k = 0; k < N; ++k) {
                const int d1 = ld1[k];
                const int vmax = q < d1 - 2 ? q : d1 - 2;
                const RT* Rk = lrt + lro[k] + q * d1;
                int v = 0;
                while (v < vmax && Rk[v + 1] <= left) ++v;
                dig[k * kSB + tid] = static_cast<uint8_t>(v);
                rem[k * kSB + tid] = static_cast<uint16_t>(q);
                left -= Rk[v];
                q -= v;
            }
        }
        R dr = 0, di = 0;
        for (int k = 0; k < p.n_diag; ++k) {
            const DevDiag g = p.diag[k];
            R f = sfactor<R>(p, g.opa, p.site[g.a].tab, dig[g.a * kSB + tid]);
            if (g.b >= 0) f *= sfactor<R>(p, g.opb, p.site[g.b].tab, dig[g.b * kSB + tid]);
            const R th = theta[g.param];
            dr += th * static_cast<R>(g.wr) * f;
            di += th * static_cast<R>(g.wi) * f;
        }
        const C xf = x[r];
        R ar = dr * xf.x - di * xf.y;
        R ai = dr * xf.y + di * xf.x;
        for (int c = 0; c < p.n_chan; ++c) {
            const DevChan ch = p.chan[c];
            const int na = dig[ch.a * kSB + tid], nb = dig[ch.b * kSB + tid];
            const int sa = na - ch.qa, sb = nb - ch.qb;
            if (sa < 0 || sa >= ld1[ch.a] - 1 || sb < 0 || sb >= ld1[ch.b] - 1) continue;
            const bool a_first = ch.a < ch.b;
            const int i = a_first ? ch.a : ch.b, j = a_first ? ch.b : ch.a;
            const int ni = a_first ? na : nb, nsi = a_first ? sa : sb;
            const int nj = a_first ? nb : na, nsj = a_first ? sb : sa;
            const int dq = nsi - ni;
            const int qi = rem[i * kSB + tid];
            int64_t drank = rt(i, qi, nsi) - rt(i, qi, ni);
            for (int k = i + 1; k < j; ++k) {
                const int qk = rem[k * kSB + tid], nk = dig[k * kSB + tid];
                drank += rt(k, qk - dq, nk) - rt(k, qk, nk);
            }
            const int qj = rem[j * kSB + tid];
            drank += rt(j, qj - dq, nsj) - rt(j, qj, nj);
            const R f = sfactor<R>(p, ch.opa, p.site[ch.a].tab, na) * sfactor<R>(p, ch.opb, p.site[ch.b].tab, nb);
            const R th = theta[ch.param] * f;
            const R cr = th * static_cast<R>(ch.wr), ci = th * static_cast<R>(ch.wi);
            const C xs = x[r + drank];
            ar += cr * xs.x - ci * xs.y;
            ai += cr * xs.y + ci * xs.x;
        }
        C out;
        out.x = ar;
        out.y = ai;
        y[r] = out;
    }
}

// Dynamic LDS of k_sector_matvec_lds for this sector (0 when it exceeds 64 KB: global-table kernel).
size_t sector_lds_bytes(const mrmf_sector_t* S, bool rt32) {
    const size_t b = (rt32 ? 4 : 8) * size_t(S->n_rt) + 8 * size_t(S->N) + 3 * size_t(S->N) * kSB;
    return b <= 65536 ? b : 0;
}

// Full-basis index F = sum_k n_k M_k of packed rows r0 .. r0 + count - 1.
__global__ __launch_bounds__(kSB) void k_sector_labels(SectorArgs a, const int64_t* __restrict__ M, int64_t r0,
                                                       int64_t count, int64_t* __restrict__ out) {
    __shared__ uint8_t dig[kMaxSites][kSB];
    __shared__ uint16_t rem[kMaxSites][kSB];
    const int tid = threadIdx.x;
    for (int64_t i = int64_t(blockIdx.x) * kSB + tid; i < count; i += int64_t(gridDim.x) * kSB) {
        unrank(a, r0 + i, dig, rem, tid);
        int64_t F = 0;
        for (int k = 0; k < a.p.N; ++k) F += int64_t(dig[k][tid]) * M[k];
        out[i] = F;
    }
}

// Packed digits of every sector state (the table the generated kernel reads instead of unranking): the
// digit of site k in w_k = bit width of d_k - 1 bits, site 0 highest, so the word of row r is the mixed-width
// concatenation n_0 n_1 .. n_{N-1}.  L is uint32_t or uint64_t.
template <typename L>
__global__ __launch_bounds__(kSB) void k_sector_pack(SectorArgs a, L* __restrict__ out) {
    for (int64_t r = int64_t(blockIdx.x) * kSB + threadIdx.x; r < a.Dr; r += int64_t(gridDim.x) * kSB) {
        int q = a.Q;
        int64_t left = r;
        L word = 0;
        for (int k = 0; k < a.p.N; ++k) {
            const int d = a.p.site[k].d;
            const int vmax = q < d - 1 ? q : d - 1;
            const int64_t* R = a.rt + a.rto[k] + int64_t(q) * (d + 1);
            int v = 0;
            while (v < vmax && R[v + 1] <= left) ++v;
            left -= R[v];
            q -= v;
            const int w = d > 1 ? 32 - __clz(d - 1) : 0;
            word = (word << w) | static_cast<L>(v);
        }
        out[r] = word;
    }
}

// Full-basis index F = sum_k n_k M_k of packed rows r0 .. r0 + count - 1 from the packed digits.
template <typename L>
__global__ __launch_bounds__(kSB) void k_sector_labels_packed(SectorArgs a, const L* __restrict__ lab,
                                                              const int64_t* __restrict__ M, int64_t r0,
                                                              int64_t count, int64_t* __restrict__ out) {
    for (int64_t i = int64_t(blockIdx.x) * kSB + threadIdx.x; i < count; i += int64_t(gridDim.x) * kSB) {
        L word = lab[r0 + i];
        int64_t F = 0;
        for (int k = a.p.N - 1; k >= 0; --k) {
            const int d = a.p.site[k].d;
            const int w = d > 1 ? 32 - __clz(d - 1) : 0;
            F += static_cast<int64_t>(word & ((L(1) << w) - 1)) * M[k];
            word >>= w;
        }
        out[i] = F;
    }
}

// Packed row of each full-basis index, or -1 when it is not a sector state (membership test).
__global__ __launch_bounds__(kSB) void k_sector_lookup(SectorArgs a, int64_t D, const int64_t* __restrict__ F,
                                                       int64_t count, int64_t* __restrict__ out) {
    for (int64_t i = int64_t(blockIdx.x) * kSB + threadIdx.x; i < count; i += int64_t(gridDim.x) * kSB) {
        int64_t f = F[i];
        if (f < 0 || f >= D) {
            out[i] = -1;
            continue;
        }
        // decode (least significant site first), then rank from site 0 with the remaining sums
        uint8_t n[kMaxSites];
        for (int k = a.p.N - 1; k >= 0; --k) {
            const int64_t d = a.p.site[k].d;
            const int64_t qq = f / d;
            n[k] = static_cast<uint8_t>(f - qq * d);
            f = qq;
        }
        int q = a.Q;
        int64_t rank = 0;
        bool ok = true;
        for (int k = 0; k < a.p.N; ++k) {
            if (n[k] > q) {
                ok = false;
                break;
            }
            rank += rtab(a, k, q, n[k]);
            q -= n[k];
        }
        out[i] = (ok && q == 0) ? rank : -1;
    }
}

// Gershgorin bounds of P H P^T: per packed row (digits from the packed-digit word when the workspace holds
// them, L = uint32_t or uint64_t, else by unranking, L = void), the diagonal entry (the real parts of the
// diagonal terms; Hermitian groups have real diagonals) -+ the sum over the sector's channels whose
// source digits are in range of |theta w f| (the channels keep the digit sum, so such a source is in the
// sector); block min / max, then one thread over the blocks.
//
// TAB: every term's contribution as a function of its two digits is tabulated in LDS when the block starts
// (diagonal terms: theta_p w_r f_a(n_a) f_b(n_b); channels: |theta_p w f_a(n_a) f_b(n_b)|, 0 where a
// source digit leaves its range), so that a row costs one LDS read per term; the tables of all terms
// together must fit kGershTab entries.  Without TAB the row evaluates the factors itself.
constexpr int kGershTab = 2048;
constexpr int kGershMaxTerms = 256;

template <typename L>
__device__ __forceinline__ void sector_row_digits(const SectorArgs& a, const void* lab, int64_t r,
                                                  uint8_t (*dig)[kSB], uint16_t (*rem)[kSB], int tid) {
    if constexpr (std::is_void_v<L>) {
        unrank(a, r, dig, rem, tid);
    } else {  // site N - 1 in the lowest bits, w_k = bit width of d_k - 1 (as k_sector_pack writes them)
        L word = static_cast<const L*>(lab)[r];
        for (int k = a.p.N - 1; k >= 0; --k) {
            const int d = a.p.site[k].d;
            const int w = d > 1 ? 32 - __clz(d - 1) : 0;
            dig[k][tid] = static_cast<uint8_t>(word & ((L(1) << w) - 1));
            word >>= w;
        }
    }
}

template <typename L, bool TAB>
__global__ __launch_bounds__(kSB) void k_sector_gershgorin(SectorArgs a, const void* __restrict__ lab,
                                                           const double* __restrict__ theta,
                                                           double* __restrict__ partial) {
    __shared__ uint8_t dig[kMaxSites][kSB];
    __shared__ uint16_t rem[kMaxSites][kSB];
    __shared__ double slo[kSB], shi[kSB];
    __shared__ double tab[TAB ? kGershTab : 1];
    __shared__ int4 td[TAB ? kGershMaxTerms : 1];  // per term: site a, site b (-1: none), d_b, table offset
    const int tid = threadIdx.x;
    const PlanArgs& p = a.p;
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
            for (int e = tid; e < n; e += kSB) {
                const int na = e / t.z, nb = e - na * t.z;
                double v;
                if (k < p.n_diag) {
                    const DevDiag g = p.diag[k];
                    double f = sfactor<double>(p, g.opa, p.site[g.a].tab, na);
                    if (g.b >= 0) f *= sfactor<double>(p, g.opb, p.site[g.b].tab, nb);
                    v = theta[g.param] * g.wr * f;
                } else {
                    const DevChan ch = p.chan[k - p.n_diag];
                    const int sa = na - ch.qa, sb = nb - ch.qb;
                    v = 0.0;
                    if (sa >= 0 && sa < p.site[ch.a].d && sb >= 0 && sb < p.site[ch.b].d)
                        v = fabs(theta[ch.param] * sfactor<double>(p, ch.opa, p.site[ch.a].tab, na) *
                                 sfactor<double>(p, ch.opb, p.site[ch.b].tab, nb)) *
                            sqrt(ch.wr * ch.wr + ch.wi * ch.wi);
                }
                tab[t.w + e] = v;
            }
        }
        __syncthreads();
    }
    double lo = __builtin_inf(), hi = -__builtin_inf();
    for (int64_t r = int64_t(blockIdx.x) * kSB + tid; r < a.Dr; r += int64_t(gridDim.x) * kSB) {
        sector_row_digits<L>(a, lab, r, dig, rem, tid);
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
                double f = sfactor<double>(p, g.opa, p.site[g.a].tab, dig[g.a][tid]);
                if (g.b >= 0) f *= sfactor<double>(p, g.opb, p.site[g.b].tab, dig[g.b][tid]);
                diag += theta[g.param] * g.wr * f;
            }
            for (int c = 0; c < p.n_chan; ++c) {
                const DevChan ch = p.chan[c];
                const int na = dig[ch.a][tid], nb = dig[ch.b][tid];
                const int sa = na - ch.qa, sb = nb - ch.qb;
                if (sa < 0 || sa >= p.site[ch.a].d || sb < 0 || sb >= p.site[ch.b].d) continue;
                const double f = sfactor<double>(p, ch.opa, p.site[ch.a].tab, na) *
                                 sfactor<double>(p, ch.opb, p.site[ch.b].tab, nb);
                rad += fabs(theta[ch.param] * f) * sqrt(ch.wr * ch.wr + ch.wi * ch.wi);
            }
        }
        lo = fmin(lo, diag - rad);
        hi = fmax(hi, diag + rad);
    }
    slo[tid] = lo;
    shi[tid] = hi;
    __syncthreads();
    if (tid == 0) {
        for (int k = 1; k < kSB; ++k) {
            lo = fmin(lo, slo[k]);
            hi = fmax(hi, shi[k]);
        }
        partial[2 * blockIdx.x] = lo;
        partial[2 * blockIdx.x + 1] = hi;
    }
}

// The same ends over count coupling vectors theta + s * stride in one pass (linear form of gersh.h).
template <typename L>
__global__ __launch_bounds__(kSB) void k_sector_gershgorin_lin(SectorArgs a, const void* __restrict__ lab,
                                                               const double* __restrict__ theta, int64_t stride,
                                                               int32_t count, double* __restrict__ partial) {
    static_assert(kSB == kLinBlock, "block size of the shared bounds code");
    __shared__ GershLinLds T;
    __shared__ uint8_t dig[kMaxSites][kSB];
    __shared__ uint16_t rem[kMaxSites][kSB];
    __shared__ double slo[kSB], shi[kSB];
    const int tid = threadIdx.x;
    const PlanArgs& p = a.p;
    gersh_lin_tables(p, [&](int op, int tab, int n) { return sfactor<double>(p, op, tab, n); }, T);
    double lo = __builtin_inf(), hi = -__builtin_inf();
    for (int64_t r = int64_t(blockIdx.x) * kSB + tid; r < a.Dr; r += int64_t(gridDim.x) * kSB) {
        sector_row_digits<L>(a, lab, r, dig, rem, tid);
        gersh_lin_row(p, T, dig, theta, stride, count, lo, hi);
    }
    gersh_block_ends(lo, hi, slo, shi, partial);
}

__global__ __launch_bounds__(kLinBlock) void k_sector_gershgorin_finalize(const double* __restrict__ partial, int nb,
                                                        double* __restrict__ out) {
    gersh_finalize_block(partial, nb, out);
}

constexpr int kSectorGershMaxGrid = 1024;

int sector_gersh_grid(int64_t n) {
    const int64_t b = (n + kSB - 1) / kSB;
    return static_cast<int>(b < kSectorGershMaxGrid ? (b < 1 ? 1 : b) : kSectorGershMaxGrid);
}

int sector_grid(int64_t n) {
    const int64_t b = (n + kSB - 1) / kSB;
    return static_cast<int>(b < 65536 ? (b < 1 ? 1 : b) : 65536);
}

template <typename R>
mrmf_status sector_matvec(mrmf_sector_t* S, const void* d_ws, const R* theta, const void* x, void* y,
                          hipStream_t s, const int32_t* skip) {
    using C = typename Cx<R>::T;
    // the kernel generated for this sector unless the plan asked for the generic kernel; the generic
    // kernels below when the sector does not qualify for it
    if (S->mode != MRMF_KERNEL_GENERIC) {
        const int dtype = sizeof(R) == 8 ? MRMF_DTYPE_Z : MRMF_DTYPE_C;
        const mrmf_status st = sector_gen_launch(S, dtype, static_cast<const unsigned char*>(d_ws) + S->off_lab, theta,
                                                 x, y, s, skip);
        if (st != MRMF_E_UNSUPPORTED) return st;
    }
    const bool rt32 = S->rt_max < (int64_t(1) << 31);
    const size_t lds = sector_lds_bytes(S, rt32);
    const dim3 grid(sector_grid(S->Dr)), block(kSB);
    if (lds == 0)
        hipLaunchKernelGGL(k_sector_matvec<R>, grid, block, 0, s, sector_args(S, d_ws), theta,
                           static_cast<const C*>(x), static_cast<C*>(y), skip);
    else if (rt32)
        hipLaunchKernelGGL((k_sector_matvec_lds<R, int32_t>), grid, block, lds, s, sector_args(S, d_ws), theta,
                           static_cast<const C*>(x), static_cast<C*>(y), skip);
    else
        hipLaunchKernelGGL((k_sector_matvec_lds<R, int64_t>), grid, block, lds, s, sector_args(S, d_ws), theta,
                           static_cast<const C*>(x), static_cast<C*>(y), skip);
    return launch_status();
}

mrmf_status check_matvec_args(const mrmf_sector_t* S, const void* d_ws, const void* theta, const void* x, void* y,
                              size_t elem) {
    if (!S || !d_ws || !x || !y || (S->n_params > 0 && !theta)) return MRMF_E_INVALID_ARG;
    if (!aligned(d_ws, 256) || !aligned(x, elem) || !aligned(y, elem)) return MRMF_E_INVALID_ARG;
    const size_t vb = size_t(S->Dr) * elem;
    if (ranges_overlap(x, vb, y, vb)) return MRMF_E_INVALID_ARG;
    return MRMF_OK;
}

}  // namespace
}  // namespace mrmf

using namespace mrmf;

extern "C" {

mrmf_status mrmf_sector_create(mrmf_plan plan, int32_t digit_sum, mrmf_sector* out) {
    if (!plan || !out) return MRMF_E_INVALID_ARG;
    *out = nullptr;
    int qmax = 0;
    for (int k = 0; k < plan->N; ++k) qmax += plan->d[k] - 1;
    if (digit_sum < 0 || digit_sum > qmax || qmax > 65535) return MRMF_E_INVALID_ARG;
    auto* S = new mrmf_sector_t;
    S->N = plan->N;
    S->Q = digit_sum;
    S->n_params = plan->n_params;
    S->hermitian = plan->hermitian;
    S->d = plan->d;
    S->M = plan->M;
    const int N = plan->N, Q = digit_sum;
    // C_k(q) for q = 0..Q (C_N(0) = 1), then R_k(q, v) = sum_{v' < v} C_{k+1}(q - v'), v = 0..d_k
    std::vector<std::vector<int64_t>> cnt(N + 1, std::vector<int64_t>(Q + 1, 0));
    cnt[N][0] = 1;
    for (int k = N - 1; k >= 0; --k)
        for (int q = 0; q <= Q; ++q) {
            int64_t c = 0;
            for (int v = 0; v < plan->d[k] && v <= q; ++v) c += cnt[k + 1][q - v];
            cnt[k][q] = c;
        }
    S->Dr = cnt[0][Q];
    std::vector<int64_t> rt, rto(N);
    for (int k = 0; k < N; ++k) {
        rto[k] = static_cast<int64_t>(rt.size());
        const int d = plan->d[k];
        for (int q = 0; q <= Q; ++q) {
            int64_t acc = 0;
            for (int v = 0; v <= d; ++v) {
                rt.push_back(acc);
                if (v < d && v <= q) acc += cnt[k + 1][q - v];
            }
        }
    }
    for (const auto& c : plan->chans)
        if (c.b >= 0 && c.qa + c.qb == 0) S->chans.push_back(c);
    S->diags = plan->diags;
    S->rt = rt;
    S->rto = rto;
    S->mode = plan->cfg[MRMF_DTYPE_Z].mode;
    S->blocks_per_cu = plan->cfg[MRMF_DTYPE_Z].blocks_per_cu;
    S->group = plan->cfg[MRMF_DTYPE_Z].group;
    S->sched = plan->cfg[MRMF_DTYPE_Z].sched;
    S->cheb_merge = plan->cfg[MRMF_DTYPE_Z].cheb_merge;
    S->cheb_fused = plan->cfg[MRMF_DTYPE_Z].cheb_fused;
    auto add_fac = [&](int site, int op) {
        for (int n = 0; n < plan->d[site]; ++n) S->tfac.push_back(local_factor_host(plan, site, op, n));
    };
    for (const auto& g : S->diags) {
        add_fac(g.a, g.opa);
        if (g.b >= 0) add_fac(g.b, g.opb);
    }
    for (const auto& c : S->chans) {
        add_fac(c.a, c.opa);
        add_fac(c.b, c.opb);
    }
    // device image
    size_t off = 0;
    auto section = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    S->off_site = section(sizeof(DevSite) * N);
    S->off_chan = section(sizeof(DevChan) * std::max<size_t>(1, S->chans.size()));
    S->off_diag = section(sizeof(DevDiag) * std::max<size_t>(1, S->diags.size()));
    S->off_val = section(sizeof(double) * plan->val.size());
    S->off_up = section(sizeof(double) * plan->up.size());
    S->off_lofs = section(sizeof(int32_t) * std::max<size_t>(1, plan->lofs.size()));
    S->off_rt = section(sizeof(int64_t) * rt.size());
    S->n_rt = static_cast<int32_t>(rt.size());
    for (int64_t v : rt) S->rt_max = std::max(S->rt_max, v);
    S->off_rto = section(sizeof(int64_t) * N);
    // packed digits of every state after the image, for the generated kernel (not in the host image: the
    // upload fills them on the device)
    const size_t img = off;
    int bits = 0;
    S->lab_w.assign(N, 0);
    for (int k = 0; k < N; ++k) {
        int w = 0;
        while ((1 << w) < plan->d[k]) ++w;
        S->lab_w[k] = w;
        bits += w;
    }
    S->lab_bytes = 0;
    if (S->mode != MRMF_KERNEL_GENERIC && bits <= 64 && S->Dr < (int64_t(1) << 28))
        S->lab_bytes = bits <= 32 ? 4 : 8;
    if (S->lab_bytes > 0) S->off_lab = section(size_t(S->lab_bytes) * size_t(S->Dr));
    S->ws_bytes = off;
    S->image.assign(img, 0);
    std::memcpy(S->image.data() + S->off_site, plan->image.data() + plan->off_site, sizeof(DevSite) * N);
    if (!S->chans.empty()) std::memcpy(S->image.data() + S->off_chan, S->chans.data(), sizeof(DevChan) * S->chans.size());
    if (!S->diags.empty()) std::memcpy(S->image.data() + S->off_diag, S->diags.data(), sizeof(DevDiag) * S->diags.size());
    std::memcpy(S->image.data() + S->off_val, plan->val.data(), sizeof(double) * plan->val.size());
    std::memcpy(S->image.data() + S->off_up, plan->up.data(), sizeof(double) * plan->up.size());
    if (!plan->lofs.empty())
        std::memcpy(S->image.data() + S->off_lofs, plan->lofs.data(), sizeof(int32_t) * plan->lofs.size());
    std::memcpy(S->image.data() + S->off_rt, rt.data(), sizeof(int64_t) * rt.size());
    std::memcpy(S->image.data() + S->off_rto, rto.data(), sizeof(int64_t) * N);
    *out = S;
    return MRMF_OK;
}

void mrmf_sector_destroy(mrmf_sector sector) { delete sector; }

mrmf_status mrmf_sector_dim(mrmf_sector sector, int64_t* dim) {
    if (!sector || !dim) return MRMF_E_INVALID_ARG;
    *dim = sector->Dr;
    return MRMF_OK;
}

mrmf_status mrmf_sector_workspace_bytes(mrmf_sector sector, size_t* bytes) {
    if (!sector || !bytes) return MRMF_E_INVALID_ARG;
    *bytes = sector->ws_bytes;
    return MRMF_OK;
}

mrmf_status mrmf_sector_upload(mrmf_sector sector, void* d_ws, size_t ws_bytes, mrmf_stream stream) {
    if (!sector || !d_ws || !aligned(d_ws, 256)) return MRMF_E_INVALID_ARG;
    if (ws_bytes < sector->ws_bytes) return MRMF_E_WORKSPACE;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const mrmf_status st =
        hip_status(hipMemcpyAsync(d_ws, sector->image.data(), sector->image.size(), hipMemcpyHostToDevice, s));
    if (st != MRMF_OK || sector->lab_bytes == 0) return st;
    // the packed digits, from the rank tables just copied
    void* lab = static_cast<unsigned char*>(d_ws) + sector->off_lab;
    if (sector->lab_bytes == 4)
        hipLaunchKernelGGL(k_sector_pack<uint32_t>, dim3(sector_grid(sector->Dr)), dim3(kSB), 0, s,
                           sector_args(sector, d_ws), static_cast<uint32_t*>(lab));
    else
        hipLaunchKernelGGL(k_sector_pack<uint64_t>, dim3(sector_grid(sector->Dr)), dim3(kSB), 0, s,
                           sector_args(sector, d_ws), static_cast<uint64_t*>(lab));
    return launch_status();
}

mrmf_status mrmf_sector_matvec_z(mrmf_sector sector, const void* d_ws, const double* d_theta, const void* d_x,
                                 void* d_y, mrmf_stream stream) {
    const mrmf_status st = check_matvec_args(sector, d_ws, d_theta, d_x, d_y, 16);
    if (st != MRMF_OK) return st;
    return sector_matvec<double>(sector, d_ws, d_theta, d_x, d_y, static_cast<hipStream_t>(stream), nullptr);
}

mrmf_status mrmf_sector_matvec_c(mrmf_sector sector, const void* d_ws, const float* d_theta, const void* d_x,
                                 void* d_y, mrmf_stream stream) {
    const mrmf_status st = check_matvec_args(sector, d_ws, d_theta, d_x, d_y, 8);
    if (st != MRMF_OK) return st;
    return sector_matvec<float>(sector, d_ws, d_theta, d_x, d_y, static_cast<hipStream_t>(stream), nullptr);
}

mrmf_status mrmf_sector_kernel_source(mrmf_sector sector, int32_t dtype, char* buf, size_t cap, size_t* len) {
    if (!sector || !len || (dtype != MRMF_DTYPE_Z && dtype != MRMF_DTYPE_C && dtype != MRMF_SOURCE_CHEB) ||
        (cap > 0 && !buf))
        return MRMF_E_INVALID_ARG;
    const bool cheb = dtype == MRMF_SOURCE_CHEB;
    const std::string src = sector_source(sector, cheb ? MRMF_DTYPE_Z : dtype, cheb);
    if (src.empty()) return MRMF_E_UNSUPPORTED;
    *len = src.size();
    if (cap > 0) {
        const size_t n = src.size() < cap - 1 ? src.size() : cap - 1;
        std::memcpy(buf, src.data(), n);
        buf[n] = '\0';
    }
    return MRMF_OK;
}

mrmf_status mrmf_sector_generated(mrmf_sector sector, int32_t dtype, int32_t* used) {
    if (!sector || !used || (dtype != MRMF_DTYPE_Z && dtype != MRMF_DTYPE_C)) return MRMF_E_INVALID_ARG;
    if (sector->mode == MRMF_KERNEL_GENERIC) {
        *used = 0;
        return MRMF_OK;
    }
    const mrmf_status st = sector_gen_prepare(sector, dtype);
    if (st != MRMF_OK && st != MRMF_E_UNSUPPORTED) return st;
    *used = st == MRMF_OK ? 1 : 0;
    return MRMF_OK;
}

mrmf_status mrmf_sector_labels(mrmf_sector sector, const void* d_ws, int64_t r0, int64_t count, int64_t* d_out,
                               void* d_scratch, size_t scratch_bytes, mrmf_stream stream) {
    if (!sector || !d_ws || !d_out || !d_scratch || r0 < 0 || count < 0 || r0 + count > sector->Dr ||
        !aligned(d_out, 8) || !aligned(d_scratch, 8))
        return MRMF_E_INVALID_ARG;
    if (scratch_bytes < sizeof(int64_t) * size_t(sector->N)) return MRMF_E_WORKSPACE;
    if (count == 0) return MRMF_OK;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const mrmf_status st = hip_status(hipMemcpyAsync(d_scratch, sector->M.data(), sizeof(int64_t) * sector->N,
                                                     hipMemcpyHostToDevice, s));
    if (st != MRMF_OK) return st;
    const unsigned char* lab = static_cast<const unsigned char*>(d_ws) + sector->off_lab;
    const dim3 grid(sector_grid(count)), block(kSB);
    const SectorArgs a = sector_args(sector, d_ws);
    const int64_t* M = static_cast<const int64_t*>(d_scratch);
    if (sector->lab_bytes == 4)
        hipLaunchKernelGGL(k_sector_labels_packed<uint32_t>, grid, block, 0, s, a,
                           reinterpret_cast<const uint32_t*>(lab), M, r0, count, d_out);
    else if (sector->lab_bytes == 8)
        hipLaunchKernelGGL(k_sector_labels_packed<uint64_t>, grid, block, 0, s, a,
                           reinterpret_cast<const uint64_t*>(lab), M, r0, count, d_out);
    else
        hipLaunchKernelGGL(k_sector_labels, grid, block, 0, s, a, M, r0, count, d_out);
    return launch_status();
}

mrmf_status mrmf_sector_lookup(mrmf_sector sector, const void* d_ws, const int64_t* d_F, int64_t count,
                               int64_t* d_out, mrmf_stream stream) {
    if (!sector || !d_ws || !d_F || !d_out || count < 0 || !aligned(d_F, 8) || !aligned(d_out, 8))
        return MRMF_E_INVALID_ARG;
    if (count == 0) return MRMF_OK;
    int64_t D = 1;
    for (int k = 0; k < sector->N; ++k) D *= sector->d[k];
    hipLaunchKernelGGL(k_sector_lookup, dim3(sector_grid(count)), dim3(kSB), 0, static_cast<hipStream_t>(stream),
                       sector_args(sector, d_ws), D, d_F, count, d_out);
    return launch_status();
}

mrmf_status mrmf_sector_lanczos_scratch_bytes(mrmf_sector sector, int32_t m, int32_t precision, size_t* bytes) {
    if (!sector) return MRMF_E_INVALID_ARG;
    return lanczos_scratch_bytes(sector->Dr, m, precision, bytes);
}

mrmf_status mrmf_sector_lanczos(mrmf_sector sector, const void* d_ws, const double* d_theta_z,
                                const float* d_theta_c, int32_t precision, int32_t m, int32_t reorth,
                                const void* d_v0, void* d_V, double* d_alpha, double* d_beta, double* d_result,
                                void* d_u, void* d_scratch, size_t scratch_bytes, mrmf_stream stream) {
    if (!sector || !d_ws || (sector->n_params > 0 && !d_theta_z) || !aligned(d_ws, 256)) return MRMF_E_INVALID_ARG;
    if (precision == MRMF_PREC_C_IN_Z && sector->n_params > 0 && !d_theta_c) return MRMF_E_INVALID_ARG;
    // P H P^T is Hermitian when H is; the Lanczos recurrence needs it (see mrmf_lanczos)
    if (!sector->hermitian) return MRMF_E_NOT_HERMITIAN;
    const MatvecOp mv_z = [&](const void* x, void* y, hipStream_t s, const int32_t* stop) {
        return sector_matvec<double>(sector, d_ws, d_theta_z, x, y, s, stop);
    };
    const MatvecOp mv_c = [&](const void* x, void* y, hipStream_t s, const int32_t* stop) {
        return sector_matvec<float>(sector, d_ws, d_theta_c, x, y, s, stop);
    };
    return lanczos_run(sector->Dr, mv_z, mv_c, precision, m, reorth, d_v0, d_V, d_alpha, d_beta, d_result, d_u,
                       d_scratch, scratch_bytes, stream);
}

mrmf_status mrmf_sector_spectral_bounds_scratch_bytes(mrmf_sector sector, size_t* bytes) {
    if (!sector || !bytes) return MRMF_E_INVALID_ARG;
    *bytes = sizeof(double) * 2 * size_t(sector_gersh_grid(sector->Dr));
    return MRMF_OK;
}

mrmf_status mrmf_sector_spectral_bounds(mrmf_sector sector, const void* d_ws, const double* d_theta, double* d_out,
                                        void* d_scratch, size_t scratch_bytes, mrmf_stream stream) {
    if (!sector || !d_ws || !d_out || !d_scratch || (sector->n_params > 0 && !d_theta)) return MRMF_E_INVALID_ARG;
    if (!sector->hermitian) return MRMF_E_NOT_HERMITIAN;
    if (!aligned(d_ws, 256) || !aligned(d_scratch, 8) || !aligned(d_out, 8)) return MRMF_E_INVALID_ARG;
    size_t need = 0;
    mrmf_sector_spectral_bounds_scratch_bytes(sector, &need);
    if (scratch_bytes < need) return MRMF_E_WORKSPACE;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int grid = sector_gersh_grid(sector->Dr);
    double* partial = static_cast<double*>(d_scratch);
    const double* theta = sector->n_params > 0 ? d_theta : partial;  // never read when there are no params
    const SectorArgs sa = sector_args(sector, d_ws);
    const void* lab = static_cast<const unsigned char*>(d_ws) + sector->off_lab;
    // per-term digit tables in LDS when they fit
    const int nt = static_cast<int>(sector->diags.size() + sector->chans.size());
    int64_t entries = 0;
    for (const auto& g : sector->diags) entries += int64_t(sector->d[g.a]) * (g.b >= 0 ? sector->d[g.b] : 1);
    for (const auto& c : sector->chans) entries += int64_t(sector->d[c.a]) * sector->d[c.b];
    const bool tab = nt <= kGershMaxTerms && entries <= kGershTab;
    const dim3 g(grid), b(kSB);
    if (sector->lab_bytes == 4) {
        if (tab) hipLaunchKernelGGL((k_sector_gershgorin<uint32_t, true>), g, b, 0, s, sa, lab, theta, partial);
        else hipLaunchKernelGGL((k_sector_gershgorin<uint32_t, false>), g, b, 0, s, sa, lab, theta, partial);
    } else if (sector->lab_bytes == 8) {
        if (tab) hipLaunchKernelGGL((k_sector_gershgorin<uint64_t, true>), g, b, 0, s, sa, lab, theta, partial);
        else hipLaunchKernelGGL((k_sector_gershgorin<uint64_t, false>), g, b, 0, s, sa, lab, theta, partial);
    } else {
        if (tab) hipLaunchKernelGGL((k_sector_gershgorin<void, true>), g, b, 0, s, sa, nullptr, theta, partial);
        else hipLaunchKernelGGL((k_sector_gershgorin<void, false>), g, b, 0, s, sa, nullptr, theta, partial);
    }
    hipLaunchKernelGGL(k_sector_gershgorin_finalize, dim3(1), dim3(kLinBlock), 0, s, partial, grid, d_out);
    return launch_status();
}

mrmf_status mrmf_sector_spectral_bounds_many(mrmf_sector sector, const void* d_ws, const double* d_theta,
                                             int64_t theta_stride, int32_t count, double* d_out, void* d_scratch,
                                             size_t scratch_bytes, mrmf_stream stream) {
    if (!sector || !d_ws || !d_out || !d_scratch || (sector->n_params > 0 && !d_theta) || count < 1 ||
        theta_stride < 0)
        return MRMF_E_INVALID_ARG;
    if (!sector->hermitian) return MRMF_E_NOT_HERMITIAN;
    if (!aligned(d_ws, 256) || !aligned(d_scratch, 8) || !aligned(d_out, 8)) return MRMF_E_INVALID_ARG;
    size_t need = 0;
    mrmf_sector_spectral_bounds_scratch_bytes(sector, &need);
    if (scratch_bytes < need) return MRMF_E_WORKSPACE;
    if (!gersh_lin_fits(sector->n_params, sector->d, sector->diags, sector->chans)) return MRMF_E_UNSUPPORTED;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int grid = sector_gersh_grid(sector->Dr);
    double* partial = static_cast<double*>(d_scratch);
    const double* theta = sector->n_params > 0 ? d_theta : partial;  // never read when there are no params
    const SectorArgs sa = sector_args(sector, d_ws);
    const void* lab = static_cast<const unsigned char*>(d_ws) + sector->off_lab;
    const dim3 g(grid), b(kSB);
    if (sector->lab_bytes == 4)
        hipLaunchKernelGGL(k_sector_gershgorin_lin<uint32_t>, g, b, 0, s, sa, lab, theta, theta_stride, count, partial);
    else if (sector->lab_bytes == 8)
        hipLaunchKernelGGL(k_sector_gershgorin_lin<uint64_t>, g, b, 0, s, sa, lab, theta, theta_stride, count, partial);
    else
        hipLaunchKernelGGL(k_sector_gershgorin_lin<void>, g, b, 0, s, sa, nullptr, theta, theta_stride, count, partial);
    hipLaunchKernelGGL(k_sector_gershgorin_finalize, dim3(1), dim3(kLinBlock), 0, s, partial, grid, d_out);
    return launch_status();
}

mrmf_status mrmf_sector_propagate_scratch_bytes(mrmf_sector sector, size_t* bytes) {
    if (!sector || !bytes) return MRMF_E_INVALID_ARG;
    *bytes = propagate_scratch_bytes(sector->Dr);
    return MRMF_OK;
}

mrmf_status mrmf_sector_propagate_z(mrmf_sector sector, const void* d_ws, const double* d_theta, int64_t theta_stride,
                                    double dt, int32_t n_steps, double e_min, double e_max, double tol,
                                    const void* d_x0, void* d_x, void* d_scratch, size_t scratch_bytes,
                                    int32_t* h_n_terms, mrmf_stream stream) {
    if (!sector || !d_ws || (sector->n_params > 0 && !d_theta) || !aligned(d_ws, 256)) return MRMF_E_INVALID_ARG;
    // the series needs the spectrum of P H P^T inside [e_min, e_max]: real, i.e. P H P^T Hermitian
    if (!sector->hermitian) return MRMF_E_NOT_HERMITIAN;
    const ThetaMatvecOp mv = [&](const double* th, const void* x, void* y, hipStream_t s) {
        return sector_matvec<double>(sector, d_ws, th, x, y, s, nullptr);
    };
    // the sector's generated kernel with the Chebyshev-step epilogue does the matvec and the update in one
    // pass; sectors on the generic kernel take the two-pass form
    const void* lab = static_cast<const unsigned char*>(d_ws) + sector->off_lab;
    const ChebStepOp step = [&](const double* th, const void* cur, void* prev, void* acc, double ea, double eb,
                                double eg, double cr, double ci, hipStream_t s) {
        return sector_gen_launch_cheb(sector, lab, th, cur, prev, acc, ea, eb, eg, cr, ci, s);
    };
    const auto fused_ready = [&]() {
        return sector->mode != MRMF_KERNEL_GENERIC && sector->cheb_fused != 0 &&
               sector_gen_prepare(sector, kSectorSlotCheb) == MRMF_OK;
    };
    return propagate_run(sector->Dr, sector->n_params, mv, &step, fused_ready, sector->cheb_merge != 0, d_theta,
                         theta_stride, dt, n_steps, e_min, e_max, tol, d_x0, d_x, d_scratch, scratch_bytes,
                         h_n_terms, static_cast<hipStream_t>(stream));
}

}  // extern "C"
