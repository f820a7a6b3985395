// Batched form: many independent lattices, each applied to a block of nvec c64 vectors, in one
// persistent launch.  Each lattice is the same target-driven gather (Sec. II) with its own digits
// (Sec. III, Eq. decode), channels and offsets (Sec. IV, Eq. sourceoffset) and ladder factors (App. A,
// App. B, App. C); the lattices only share the launch.
//
// Layout.  Lattice b's vectors are stored row-major as [D_b][nvec] at element offset off_b of X and Y
// (row F holds its nvec amplitudes contiguously, so one row is 8 * nvec bytes); offsets are multiples
// of 32 elements.
//
// Shared input (parameter sweeps: the same vectors under many couplings): every lattice reads block 0 of X,
// and the items are numbered tile by tile across the lattices instead of lattice by lattice.
//
// Work.  For a launch shape (R_max, block B), lattice b's rows are cut into tiles spanned by its low
// sites (T_b = prod of the low d_i, the largest such product <= R_max), and an item is the P = max(1,
// B / T_b) consecutive tiles that one block holds in LDS at a time (rows stored vector-major, so that
// consecutive threads read consecutive 8-byte words).  Items are numbered lattice by lattice.  Three
// schedules: runs - block v of the grid takes the contiguous item range [v I / G, (v+1) I / G), v chosen
// so that the blocks of one XCD (block b runs on XCD b mod 8) hold neighbouring ranges; windows - the
// grid sweeps windows of G consecutive items, the blocks of one XCD taking one eighth of each window side
// by side, so that the items an XCD works on at one time are neighbours and the gathers of one item find
// the rows its neighbours have just read in the XCD's L2 (at the price of reloading a lattice's
// descriptors whenever a block moves to another lattice); XCD chunks - XCD x sweeps the x-th eighth of
// the items with its blocks side by side, so that its L2 also holds the rows it read further back.  Every thread owns rows of the item; for each
// row it decodes the digits once into LDS, then for every channel forms the coefficient from the
// per-site factor tables (zero where a source digit is inadmissible, App. A) and, where it is nonzero,
// reads the nvec source amplitudes of row F - Delta: from LDS when both sites of the channel lie in the
// tile (the source is then in the same tile), else from global memory.  A nonzero factor means both
// source digits are in range, so no read leaves the lattice.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "mrmf_internal.h"

namespace mrmf {
namespace {

constexpr int kBatchMaxLattices = 2048;
constexpr int kBatchMaxSites = 32;
constexpr int kBatchMaxBlock = 512;
constexpr int kBatchPoolMax = 2048;    // factor-table entries of one lattice (LDS)
constexpr int kBatchTileWords = 4096;  // 8-byte words of the LDS tile (32 KB): at most 4096 / nvec rows
constexpr int kBatchRmaxCands = 4;     // tile-row limits R_max = (64, 128, 256, 512) * 8 / nvec
constexpr int kBatchMaxTerms = 128;    // terms (channels + diagonal) of one lattice, held in LDS
constexpr int kBatchMaxParams = 128;   // couplings of one lattice, held in LDS
constexpr int kBatchGather = 5;        // global-memory channels whose gathers are issued together (124 VGPRs:
                                       // still 4 waves per SIMD; 6 or 8 fall to 3 or 2 and run slower)

struct alignas(16) BLat {
    int32_t N, n_chan, n_diag, theta_off;
    int32_t D, chan_off, diag_off, site_off;
    int32_t pool_off, pool_n, n_params, pad1;
    int64_t x_off, pad2;
    int32_t tile_rows[kBatchRmaxCands];   // T_b for each R_max candidate
    int32_t tile_sites[kBatchRmaxCands];  // number of low sites spanning T_b
    int32_t n_local[kBatchRmaxCands];     // channels whose source lies in the tile (a prefix of the list)
};
static_assert(sizeof(BLat) == 112, "BLat layout");

struct alignas(16) BSite {
    int32_t d, pad;
    uint64_t magic;  // ceil(2^64 / d)
};
static_assert(sizeof(BSite) == 16, "BSite layout");

// One term: coefficient theta[param] * (wr + i wi) * pool[ta + n_a] * pool[tb + n_b]; source F - delta.
// A one-site term has b = -1 (its second factor is the pool's 1.0 entry at tb, digit 0).  low = number of
// low sites a tile must span for the term's sites to lie in it.
struct alignas(16) BTerm {
    int32_t a, b, ta, tb;
    int32_t param, delta, low, pad;
    float wr, wi, pad1, pad2;
};
static_assert(sizeof(BTerm) == 48, "BTerm layout");

struct BatchArgs {
    const BLat* lat;
    const BSite* site;
    const BTerm* term;   // channels and diagonal terms of every lattice
    const float* pool;   // factor tables of every lattice
    int32_t n_lat;
    int32_t all_real;
    int32_t shared;  // every lattice reads its input rows from the one block at the start of X; items tile-major
};

__device__ __forceinline__ uint32_t umulhi_div(uint32_t n, uint64_t magic) {
    return static_cast<uint32_t>(__umul64hi(magic, static_cast<uint64_t>(n)));
}

// The NV amplitudes of one row (NV * 8 contiguous bytes; 16-byte aligned when NV >= 2) in 16-byte loads
// and stores where the row allows it.
template <int NV>
__device__ __forceinline__ void load_row(const float2* __restrict__ src, float2 (&v)[NV]) {
    if constexpr (NV == 1) {
        v[0] = src[0];
    } else {
        const float4* s4 = reinterpret_cast<const float4*>(src);
#pragma unroll
        for (int q = 0; q < NV / 2; ++q) {
            const float4 w = s4[q];
            v[2 * q] = make_float2(w.x, w.y);
            v[2 * q + 1] = make_float2(w.z, w.w);
        }
    }
}

template <int NV>
__device__ __forceinline__ void store_row(float2* __restrict__ dst, const float (&re)[NV], const float (&im)[NV]) {
    if constexpr (NV == 1) {
        dst[0] = make_float2(re[0], im[0]);
    } else {
        float4* d4 = reinterpret_cast<float4*>(dst);
#pragma unroll
        for (int q = 0; q < NV / 2; ++q) d4[q] = make_float4(re[2 * q], im[2 * q], re[2 * q + 1], im[2 * q + 1]);
    }
}

template <int NV, bool CPLX>
__global__ __launch_bounds__(kBatchMaxBlock) void k_batch(BatchArgs A, const float* __restrict__ theta_all,
                                                        const float2* __restrict__ X, float2* __restrict__ Y,
                                                        int32_t rc, int32_t sched) {
    constexpr int kRows = kBatchTileWords / NV;
    __shared__ int32_t ibeg[kBatchMaxLattices + 1];
    __shared__ float pool[kBatchPoolMax];
    __shared__ uint8_t dig[kBatchMaxSites][kBatchMaxBlock];
    __shared__ float2 xt[NV][kRows];
    __shared__ BTerm tl[kBatchMaxTerms];  // the current lattice's diagonal terms, then its channels
    __shared__ BSite sl[kBatchMaxSites];
    __shared__ float thl[kBatchMaxParams];
    const int tid = threadIdx.x, B = blockDim.x;
    // items: ibeg[b] = sum over b' < b of ceil(D_b' / (P_b' T_b')); counts in parallel, then a serial scan
    // over LDS by thread 0 (n <= 2048)
    for (int b = tid; b < A.n_lat; b += B) {
        const int32_t T = A.lat[b].tile_rows[rc];
        const int32_t rows = T >= B ? T : (B / T) * T;
        ibeg[b + 1] = (A.lat[b].D + rows - 1) / rows;
    }
    __syncthreads();
    if (tid == 0) {
        int32_t s = 0;
        ibeg[0] = 0;
        for (int b = 1; b <= A.n_lat; ++b) {
            s += ibeg[b];
            ibeg[b] = s;
        }
    }
    __syncthreads();
    const int64_t I = ibeg[A.n_lat];
    const unsigned G = gridDim.x, bid = blockIdx.x;
    const unsigned v = (G % 8u == 0u) ? (bid % 8u) * (G / 8u) + bid / 8u : bid;
    int32_t i0, i1, step;
    if (sched == 1) {  // windows
        i0 = static_cast<int32_t>(v);
        i1 = static_cast<int32_t>(I);
        step = static_cast<int32_t>(G);
    } else if (sched == 2) {  // XCD x sweeps the x-th eighth of the items with its blocks side by side
        const unsigned nx = (G % 8u == 0u) ? 8u : 1u, xcd = bid % nx;
        const int64_t C = (I + nx - 1) / nx;
        i0 = static_cast<int32_t>(xcd * C + bid / nx);
        i1 = static_cast<int32_t>((xcd + 1) * C < I ? (xcd + 1) * C : I);
        step = static_cast<int32_t>(G / nx);
    } else {  // runs
        i0 = static_cast<int32_t>(int64_t(v) * I / G);
        i1 = static_cast<int32_t>(int64_t(v + 1) * I / G);
        step = 1;
    }
    // the current lattice's descriptor, kept in scalar registers (every field is block-uniform)
    int lb = -1;
    int32_t N = 0, n_chan = 0, n_diag = 0, D = 0, rows = 1, ks = 0, n_loc = 0;
    const float2* xb = X;
    float2* yb = Y;
    int b = 0;
    const bool shared = A.shared != 0;
    if (!shared) {
        int lo = 0, hi = A.n_lat - 1;  // last lattice with ibeg[b] <= i0
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (ibeg[mid] <= i0) lo = mid; else hi = mid - 1;
        }
        b = lo;
    }
    for (int32_t it = i0; it < i1; it += step) {
        // shared input: every lattice has the same tiles; item it is tile it / n of lattice it mod n, so the
        // items worked on together read the same input rows
        int32_t li;
        if (shared) {
            b = it % A.n_lat;
            li = it / A.n_lat;
        } else {
            while (it >= ibeg[b + 1]) ++b;
            li = it - ibeg[b];
        }
        b = __builtin_amdgcn_readfirstlane(b);
        li = __builtin_amdgcn_readfirstlane(li);
        __syncthreads();  // every thread is done with the previous item's tile (and tables)
        if (b != lb) {
            const BLat* L = A.lat + b;
            N = __builtin_amdgcn_readfirstlane(L->N);
            n_chan = __builtin_amdgcn_readfirstlane(L->n_chan);
            n_diag = __builtin_amdgcn_readfirstlane(L->n_diag);
            D = __builtin_amdgcn_readfirstlane(L->D);
            const int32_t T = __builtin_amdgcn_readfirstlane(L->tile_rows[rc]);
            ks = __builtin_amdgcn_readfirstlane(L->tile_sites[rc]);
            n_loc = __builtin_amdgcn_readfirstlane(L->n_local[rc]);
            rows = T >= B ? T : (B / T) * T;
            const int64_t xo = L->x_off;
            xb = shared ? X : X + xo;
            yb = Y + xo;
            const int32_t po = __builtin_amdgcn_readfirstlane(L->pool_off), pn = __builtin_amdgcn_readfirstlane(L->pool_n);
            for (int k = tid; k < pn; k += B) pool[k] = A.pool[po + k];
            // descriptors into LDS: diagonal terms then channels (stored contiguously), sites, couplings
            const int32_t t0 = L->diag_off, nt = n_diag + n_chan, s0 = L->site_off, th0 = L->theta_off;
            for (int k = tid; k < nt; k += B) tl[k] = A.term[t0 + k];
            for (int k = tid; k < N; k += B) sl[k] = A.site[s0 + k];
            for (int k = tid; k < A.lat[b].n_params; k += B) thl[k] = theta_all[th0 + k];
            lb = b;
            __syncthreads();
        }
        const int32_t r0 = li * rows;
        const int32_t nr = r0 + rows < D ? rows : D - r0;
        for (int32_t r = tid; r < nr; r += B) {
            float2 v[NV];
            load_row<NV>(xb + int64_t(r0 + r) * NV, v);
#pragma unroll
            for (int q = 0; q < NV; ++q) xt[q][r] = v[q];
        }
        __syncthreads();
        for (int32_t r = tid; r < nr; r += B) {
            const int32_t F = r0 + r;
            // digits, least significant site first (Eq. decode)
            uint32_t f = static_cast<uint32_t>(F);
            for (int i = N - 1; i >= 0; --i) {
                const BSite s = sl[i];
                const uint32_t q = umulhi_div(f, s.magic);
                dig[i][tid] = static_cast<uint8_t>(f - q * static_cast<uint32_t>(s.d));
                f = q;
            }
            float ar[NV], ai[NV];
            float dr = 0.f, di = 0.f;
            for (int k = 0; k < n_diag; ++k) {
                const BTerm t = tl[k];
                const float fa = pool[t.ta + dig[t.a][tid]] * (t.b >= 0 ? pool[t.tb + dig[t.b][tid]] : 1.f);
                const float c = thl[t.param] * fa;
                dr += c * t.wr;
                if (CPLX) di += c * t.wi;
            }
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                const float2 s = xt[q][r];
                ar[q] = dr * s.x;
                ai[q] = dr * s.y;
                if (CPLX) {
                    ar[q] -= di * s.y;
                    ai[q] += di * s.x;
                }
            }
            // channels whose sites both lie in the tile (the first n_loc): the source row is in LDS
            // (Eq. sourceoffset)
            for (int k = 0; k < n_loc; ++k) {
                const BTerm t = tl[n_diag + k];
                const float fa = pool[t.ta + dig[t.a][tid]] * (t.b >= 0 ? pool[t.tb + dig[t.b][tid]] : 1.f);
                if (fa == 0.f) continue;  // an inadmissible source digit has factor 0 (App. A)
                const float c = thl[t.param] * fa;
                const float cr = c * t.wr, ci = CPLX ? c * t.wi : 0.f;
                const int32_t rs = r - t.delta;
#pragma unroll
                for (int q = 0; q < NV; ++q) {
                    const float2 s = xt[q][rs];
                    ar[q] += cr * s.x;
                    ai[q] += cr * s.y;
                    if (CPLX) {
                        ar[q] -= ci * s.y;
                        ai[q] += ci * s.x;
                    }
                }
            }
            // the others read global memory, kBatchGather channels at a time: every gather of a group is
            // issued (masked where the factor is 0) before any of them is used
            for (int k0 = n_loc; k0 < n_chan; k0 += kBatchGather) {
                float cr[kBatchGather], ci[kBatchGather];
                float2 v[kBatchGather][NV];
#pragma unroll
                for (int u = 0; u < kBatchGather; ++u) {
                    cr[u] = 0.f;
                    ci[u] = 0.f;
                    if (k0 + u < n_chan) {
                        const BTerm t = tl[n_diag + k0 + u];
                        const float fa =
                            pool[t.ta + dig[t.a][tid]] * (t.b >= 0 ? pool[t.tb + dig[t.b][tid]] : 1.f);
                        const float c = thl[t.param] * fa;
                        cr[u] = c * t.wr;
                        ci[u] = CPLX ? c * t.wi : 0.f;
                        if (fa != 0.f) {  // a nonzero factor: both source digits in range (App. A)
                            load_row<NV>(xb + int64_t(F - t.delta) * NV, v[u]);
                            continue;
                        }
                    }
#pragma unroll
                    for (int q = 0; q < NV; ++q) v[u][q] = make_float2(0.f, 0.f);
                }
#pragma unroll
                for (int u = 0; u < kBatchGather; ++u) {
#pragma unroll
                    for (int q = 0; q < NV; ++q) {
                        const float2 s = v[u][q];
                        ar[q] += cr[u] * s.x;
                        ai[q] += cr[u] * s.y;
                        if (CPLX) {
                            ar[q] -= ci[u] * s.y;
                            ai[q] += ci[u] * s.x;
                        }
                    }
                }
            }
            store_row<NV>(yb + int64_t(F) * NV, ar, ai);
        }
    }
}

// Linear combination of parameter-group products: Y_k[i] = sum_p theta[k][p] G_p[i] for k < K, i < n (c64
// entries, real couplings).  A thread holds the P entries G_p[i] of its element in registers and writes
// every Y_k[i]; the couplings of the sweep sit in LDS.  Bound by the writes of the K outputs.
constexpr int kCombMaxP = 16;
constexpr int kCombTheta = 4096;  // couplings held in LDS at a time (16 KB)
constexpr int kCombBlock = 256;

template <int P>
__global__ __launch_bounds__(kCombBlock) void k_sweep_combine(const float* __restrict__ theta, int32_t K,
                                                              int64_t n, const float2* __restrict__ G,
                                                              int64_t g_stride, float2* __restrict__ Y,
                                                              int64_t y_stride) {
    __shared__ float th[kCombTheta];  // a chunk of the sweep's couplings, rows of P
    const int64_t i = int64_t(blockIdx.x) * kCombBlock + threadIdx.x;
    float2 g[P];
#pragma unroll
    for (int p = 0; p < P; ++p) g[p] = i < n ? G[p * g_stride + i] : make_float2(0.f, 0.f);
    const int kc = kCombTheta / P;  // sweep rows per chunk
    for (int k0 = 0; k0 < K; k0 += kc) {
        const int kn = K - k0 < kc ? K - k0 : kc;
        __syncthreads();
        for (int e = threadIdx.x; e < kn * P; e += kCombBlock) th[e] = theta[int64_t(k0) * P + e];
        __syncthreads();
        if (i < n)
            for (int k = 0; k < kn; ++k) {
                float yr = 0.f, yi = 0.f;
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    const float t = th[k * P + p];
                    yr += t * g[p].x;
                    yi += t * g[p].y;
                }
                Y[(k0 + k) * y_stride + i] = make_float2(yr, yi);
            }
    }
}

template <int P>
void launch_combine(const float* theta, int32_t K, int64_t n, const float2* G, int64_t gs, float2* Y, int64_t ys,
                    hipStream_t s) {
    const int64_t grid = (n + kCombBlock - 1) / kCombBlock;
    hipLaunchKernelGGL(k_sweep_combine<P>, dim3(static_cast<unsigned>(grid)), dim3(kCombBlock), 0, s, theta, K, n,
                       G, gs, Y, ys);
}

template <int NV>
void* batch_kernel_ptr(bool cplx) {
    return cplx ? reinterpret_cast<void*>(&k_batch<NV, true>) : reinterpret_cast<void*>(&k_batch<NV, false>);
}

void* batch_kernel(int nvec, bool cplx) {
    switch (nvec) {
        case 1: return batch_kernel_ptr<1>(cplx);
        case 2: return batch_kernel_ptr<2>(cplx);
        case 4: return batch_kernel_ptr<4>(cplx);
        default: return batch_kernel_ptr<8>(cplx);
    }
}

// Factor table <n|O|n - q> at target digit n (0 where the source digit n - q is outside 0..d-1).
void factor_table(const mrmf_plan_t* p, int site, int op, std::vector<float>& out) {
    for (int n = 0; n < p->d[site]; ++n) out.push_back(static_cast<float>(local_factor_host(p, site, op, n)));
}

// Launch shapes tried by the autotuner: (R_max candidate index, block threads).
struct Shape {
    int32_t rc, block;
};
const Shape kShapes[] = {{1, 128}, {2, 128}, {2, 256}, {3, 256}, {3, 512}, {0, 64}, {1, 256}, {0, 128}};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

int32_t rmax_of(int rc, int nvec) { return (64 << rc) * 8 / nvec; }

}  // namespace
}  // namespace mrmf

struct mrmf_batch_t {
    int32_t n = 0, nvec = 0;
    std::vector<int64_t> off;      // element offset of each lattice's block
    std::vector<int32_t> th_off;   // n + 1
    int64_t total = 0;             // elements, padded
    bool all_real = true;
    std::vector<unsigned char> image;
    size_t off_lat = 0, off_site = 0, off_term = 0, off_pool = 0, ws_bytes = 0;
    int32_t rc = 2, block = 256;  // R_max candidate index and block threads
    int32_t sched = 0;            // MRMF_BATCH_SCHED_*
    int32_t grid = 0;
    bool shared = false;                     // mrmf_batch_share_input
    std::vector<std::vector<int32_t>> dims;  // local dimensions of each lattice
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~mrmf_batch_t() {
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
    }
};

namespace {

mrmf::BatchArgs batch_args(const mrmf_batch_t* b, const void* d_ws) {
    const unsigned char* w = static_cast<const unsigned char*>(d_ws);
    mrmf::BatchArgs a;
    a.lat = reinterpret_cast<const mrmf::BLat*>(w + b->off_lat);
    a.site = reinterpret_cast<const mrmf::BSite*>(w + b->off_site);
    a.term = reinterpret_cast<const mrmf::BTerm*>(w + b->off_term);
    a.pool = reinterpret_cast<const float*>(w + b->off_pool);
    a.n_lat = b->n;
    a.all_real = b->all_real ? 1 : 0;
    a.shared = b->shared ? 1 : 0;
    return a;
}

int batch_grid(const mrmf_batch_t* b) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    // two resident blocks per CU (LDS: tile 32 KB, item table 8 KB, digits, factor pool, descriptors)
    const int per_cu = 2;
    return cus * per_cu;
}

mrmf_status launch(mrmf_batch_t* b, const void* d_ws, const float* theta, const void* X, void* Y, hipStream_t s) {
    const mrmf::BatchArgs a = batch_args(b, d_ws);
    void* fn = mrmf::batch_kernel(b->nvec, !b->all_real);
    const int grid = batch_grid(b);
    b->grid = grid;
    int32_t rc = b->rc, sched = b->sched;
    const float2* xp = static_cast<const float2*>(X);
    float2* yp = static_cast<float2*>(Y);
    void* args[] = {const_cast<mrmf::BatchArgs*>(&a), &theta, &xp, &yp, &rc, &sched};
    return mrmf::hip_status(hipLaunchKernel(fn, dim3(grid), dim3(b->block), args, 0, s));
}

mrmf_status check_call(const mrmf_batch_t* b, const void* d_ws, const float* th, const void* X, const void* Y) {
    if (!b || !d_ws || !th || !X || !Y) return MRMF_E_INVALID_ARG;
    const size_t al = b->nvec >= 2 ? 16 : 8;  // rows are moved in 16-byte words when they hold two or more
    if (!mrmf::aligned(d_ws, 256) || !mrmf::aligned(X, al) || !mrmf::aligned(Y, al)) return MRMF_E_INVALID_ARG;
    const size_t bytes = size_t(b->total) * 8;
    const size_t x_bytes = b->shared ? size_t(b->off.size() > 1 ? b->off[1] : b->total) * 8 : bytes;
    if (mrmf::ranges_overlap(X, x_bytes, Y, bytes)) return MRMF_E_INVALID_ARG;
    return MRMF_OK;
}

}  // namespace

extern "C" {

mrmf_status mrmf_batch_create(int32_t n, const mrmf_plan* plans, int32_t nvec, mrmf_batch* out) {
    using namespace mrmf;
    if (!out) return MRMF_E_INVALID_ARG;
    *out = nullptr;
    if (n < 1 || n > kBatchMaxLattices || !plans) return MRMF_E_INVALID_ARG;
    if (nvec != 1 && nvec != 2 && nvec != 4 && nvec != 8) return MRMF_E_INVALID_ARG;
    auto* b = new (std::nothrow) mrmf_batch_t();
    if (!b) return MRMF_E_INVALID_ARG;
    b->n = n;
    b->nvec = nvec;
    std::vector<BLat> lats(n);
    std::vector<BSite> sites;
    std::vector<BTerm> terms;
    std::vector<float> pool;
    int64_t off = 0;
    int32_t th = 0;
    for (int i = 0; i < n; ++i) {
        const mrmf_plan_t* p = plans[i];
        if (!p || p->N > kBatchMaxSites || p->D >= (int64_t(1) << 31) / 2 / nvec || p->n_params > kBatchMaxParams ||
            p->chans.size() + p->diags.size() > size_t(kBatchMaxTerms)) {
            delete b;
            return p ? MRMF_E_UNSUPPORTED : MRMF_E_INVALID_ARG;
        }
        BLat& L = lats[i];
        for (int rc = 0; rc < kBatchRmaxCands; ++rc) {  // tiles spanned by the low sites, <= R_max rows
            const int64_t rmax = rmax_of(rc, nvec);
            int64_t T = 1;
            int k = 0;
            while (k < p->N && T * p->d[p->N - 1 - k] <= rmax) T *= p->d[p->N - 1 - k++];
            L.tile_rows[rc] = static_cast<int32_t>(T);
            L.tile_sites[rc] = k;
        }
        b->dims.emplace_back(p->d.begin(), p->d.end());
        L.N = p->N;
        L.n_params = p->n_params;
        L.D = static_cast<int32_t>(p->D);
        L.theta_off = th;
        L.x_off = off;
        L.site_off = static_cast<int32_t>(sites.size());
        for (int s = 0; s < p->N; ++s) {
            BSite bs{};
            bs.d = p->d[s];
            bs.magic = ~uint64_t(0) / uint64_t(p->d[s]) + 1;
            sites.push_back(bs);
        }
        // factor pool of this lattice: entry 0 is 1.0 (second factor of a one-site term)
        std::vector<float> lp{1.0f};
        auto table = [&](int s, int op) {
            const int at = static_cast<int>(lp.size());
            factor_table(p, s, op, lp);
            return at;
        };
        auto add_term = [&](int a, int opa, int bsite, int opb, int param, double wr, double wi, int64_t delta) {
            BTerm t{};
            t.a = a;
            t.ta = table(a, opa);
            t.b = bsite;
            t.tb = bsite >= 0 ? table(bsite, opb) : 0;
            t.param = param;
            t.delta = static_cast<int32_t>(delta);
            t.low = p->N - (bsite >= 0 && bsite < a ? bsite : a);
            t.wr = static_cast<float>(wr);
            t.wi = static_cast<float>(wi);
            if (wi != 0.0) b->all_real = false;
            terms.push_back(t);
        };
        L.diag_off = static_cast<int32_t>(terms.size());
        for (const auto& g : p->diags) add_term(g.a, g.opa, g.b, g.opb, g.param, g.wr, g.wi, 0);
        L.n_diag = static_cast<int32_t>(p->diags.size());
        L.chan_off = static_cast<int32_t>(terms.size());
        for (const auto& c : p->chans) add_term(c.a, c.opa, c.b, c.opb, c.param, c.wr, c.wi, c.delta);
        L.n_chan = static_cast<int32_t>(p->chans.size());
        // channels by the number of low sites a tile must span (stable), so that for every tile size the
        // channels whose source lies in the tile are a prefix of the list
        std::stable_sort(terms.begin() + L.chan_off, terms.end(),
                         [](const BTerm& u, const BTerm& v) { return u.low < v.low; });
        for (int rc = 0; rc < kBatchRmaxCands; ++rc) {
            int32_t nl = 0;
            for (size_t k = L.chan_off; k < terms.size(); ++k) nl += terms[k].low <= L.tile_sites[rc];
            L.n_local[rc] = nl;
        }
        if (lp.size() > size_t(kBatchPoolMax)) {
            delete b;
            return MRMF_E_UNSUPPORTED;
        }
        L.pool_off = static_cast<int32_t>(pool.size());
        L.pool_n = static_cast<int32_t>(lp.size());
        pool.insert(pool.end(), lp.begin(), lp.end());
        b->off.push_back(off);
        b->th_off.push_back(th);
        off += (p->D * nvec + 31) / 32 * 32;
        th += p->n_params;
    }
    b->th_off.push_back(th);
    b->total = off;
    if (off * 8 >= (int64_t(1) << 62)) {
        delete b;
        return MRMF_E_OVERFLOW;
    }
    size_t o = 0;
    b->off_lat = o;
    o = align_up(o + sizeof(BLat) * lats.size(), 256);
    b->off_site = o;
    o = align_up(o + sizeof(BSite) * sites.size(), 256);
    b->off_term = o;
    o = align_up(o + sizeof(BTerm) * std::max<size_t>(1, terms.size()), 256);
    b->off_pool = o;
    o = align_up(o + sizeof(float) * pool.size(), 256);
    b->ws_bytes = o;
    b->image.assign(o, 0);
    std::memcpy(b->image.data() + b->off_lat, lats.data(), sizeof(BLat) * lats.size());
    std::memcpy(b->image.data() + b->off_site, sites.data(), sizeof(BSite) * sites.size());
    if (!terms.empty()) std::memcpy(b->image.data() + b->off_term, terms.data(), sizeof(BTerm) * terms.size());
    std::memcpy(b->image.data() + b->off_pool, pool.data(), sizeof(float) * pool.size());
    *out = b;
    return MRMF_OK;
}

void mrmf_batch_destroy(mrmf_batch batch) { delete batch; }

mrmf_status mrmf_batch_total_elems(mrmf_batch b, int64_t* elems) {
    if (!b || !elems) return MRMF_E_INVALID_ARG;
    *elems = b->total;
    return MRMF_OK;
}

mrmf_status mrmf_batch_offsets(mrmf_batch b, int64_t* out) {
    if (!b || !out) return MRMF_E_INVALID_ARG;
    std::memcpy(out, b->off.data(), sizeof(int64_t) * b->n);
    return MRMF_OK;
}

mrmf_status mrmf_batch_theta_offsets(mrmf_batch b, int32_t* out) {
    if (!b || !out) return MRMF_E_INVALID_ARG;
    std::memcpy(out, b->th_off.data(), sizeof(int32_t) * (b->n + 1));
    return MRMF_OK;
}

mrmf_status mrmf_batch_workspace_bytes(mrmf_batch b, size_t* bytes) {
    if (!b || !bytes) return MRMF_E_INVALID_ARG;
    *bytes = b->ws_bytes;
    return MRMF_OK;
}

mrmf_status mrmf_batch_upload(mrmf_batch b, void* d_ws, size_t ws_bytes, mrmf_stream stream) {
    if (!b || !d_ws || !mrmf::aligned(d_ws, 256)) return MRMF_E_INVALID_ARG;
    if (ws_bytes < b->ws_bytes) return MRMF_E_WORKSPACE;
    return mrmf::hip_status(hipMemcpyAsync(d_ws, b->image.data(), b->ws_bytes, hipMemcpyHostToDevice,
                                           static_cast<hipStream_t>(stream)));
}

mrmf_status mrmf_batch_matvec_c(mrmf_batch b, const void* d_ws, const float* d_theta_all, const void* d_X,
                                void* d_Y, mrmf_stream stream) {
    const mrmf_status st = check_call(b, d_ws, d_theta_all, d_X, d_Y);
    if (st != MRMF_OK) return st;
    return launch(b, d_ws, d_theta_all, d_X, d_Y, static_cast<hipStream_t>(stream));
}

mrmf_status mrmf_batch_graph_capture(mrmf_batch b, const void* d_ws, const float* d_theta_all, const void* d_X,
                                     void* d_Y, mrmf_stream stream) {
    mrmf_status st = check_call(b, d_ws, d_theta_all, d_X, d_Y);
    if (st != MRMF_OK) return st;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    if (b->exec) {
        hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return MRMF_E_HIP;
    st = launch(b, d_ws, d_theta_all, d_X, d_Y, s);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &g);
    if (st != MRMF_OK || e != hipSuccess || !g) {
        if (g) hipGraphDestroy(g);
        return st != MRMF_OK ? st : MRMF_E_HIP;
    }
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        hipGraphDestroy(g);
        return MRMF_E_HIP;
    }
    b->graph = g;
    b->exec = ex;
    return MRMF_OK;
}

mrmf_status mrmf_batch_graph_launch(mrmf_batch b, mrmf_stream stream) {
    if (!b || !b->exec) return MRMF_E_INVALID_ARG;
    return mrmf::hip_status(hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)));
}

mrmf_status mrmf_batch_share_input(mrmf_batch b, int32_t on) {
    if (!b || (on != 0 && on != 1)) return MRMF_E_INVALID_ARG;
    if (on)
        for (const auto& d : b->dims)
            if (d != b->dims[0]) return MRMF_E_UNSUPPORTED;
    b->shared = on != 0;
    return MRMF_OK;
}

mrmf_status mrmf_sweep_combine_c(const float* d_theta, int32_t K, int32_t P, int64_t n, const void* d_G,
                                 int64_t g_stride, void* d_Y, int64_t y_stride, mrmf_stream stream) {
    using namespace mrmf;
    if (!d_theta || !d_G || !d_Y || K < 1 || P < 1 || P > kCombMaxP || n < 1 || g_stride < n || y_stride < n)
        return MRMF_E_INVALID_ARG;
    if (n >= (int64_t(1) << 31) * kCombBlock) return MRMF_E_INVALID_ARG;
    if (!aligned(d_G, 8) || !aligned(d_Y, 8) || !aligned(d_theta, 4)) return MRMF_E_INVALID_ARG;
    const size_t gb = size_t(g_stride) * (P - 1) * 8 + size_t(n) * 8, yb = size_t(y_stride) * (K - 1) * 8 + size_t(n) * 8;
    if (ranges_overlap(d_G, gb, d_Y, yb)) return MRMF_E_INVALID_ARG;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const auto* G = static_cast<const float2*>(d_G);
    auto* Y = static_cast<float2*>(d_Y);
    switch (P) {
#define MRMF_COMB_CASE(q) \
    case q: launch_combine<q>(d_theta, K, n, G, g_stride, Y, y_stride, s); break;
        MRMF_COMB_CASE(1) MRMF_COMB_CASE(2) MRMF_COMB_CASE(3) MRMF_COMB_CASE(4) MRMF_COMB_CASE(5) MRMF_COMB_CASE(6)
        MRMF_COMB_CASE(7) MRMF_COMB_CASE(8) MRMF_COMB_CASE(9) MRMF_COMB_CASE(10) MRMF_COMB_CASE(11)
        MRMF_COMB_CASE(12) MRMF_COMB_CASE(13) MRMF_COMB_CASE(14) MRMF_COMB_CASE(15) MRMF_COMB_CASE(16)
#undef MRMF_COMB_CASE
        default: return MRMF_E_INVALID_ARG;
    }
    return launch_status();
}

mrmf_status mrmf_batch_set_shape(mrmf_batch b, int32_t tile_rows_max, int32_t block_threads) {
    if (!b || block_threads < 64 || block_threads > mrmf::kBatchMaxBlock || block_threads % 64 != 0 ||
        block_threads > mrmf::kBatchTileWords / b->nvec)
        return MRMF_E_INVALID_ARG;
    int rc = -1;
    for (int k = 0; k < mrmf::kBatchRmaxCands; ++k)
        if (mrmf::rmax_of(k, b->nvec) == tile_rows_max) rc = k;
    if (rc < 0) return MRMF_E_INVALID_ARG;
    b->rc = rc;
    b->block = block_threads;
    return MRMF_OK;
}

mrmf_status mrmf_batch_set_schedule(mrmf_batch b, int32_t sched) {
    if (!b || (sched != MRMF_BATCH_SCHED_RUNS && sched != MRMF_BATCH_SCHED_WINDOWS &&
               sched != MRMF_BATCH_SCHED_XCD_CHUNK))
        return MRMF_E_INVALID_ARG;
    b->sched = sched;
    return MRMF_OK;
}

mrmf_status mrmf_batch_get_shape(mrmf_batch b, int32_t* out) {
    if (!b || !out) return MRMF_E_INVALID_ARG;
    out[0] = mrmf::rmax_of(b->rc, b->nvec);
    out[1] = b->block;
    out[2] = b->sched;
    out[3] = batch_grid(b);
    return MRMF_OK;
}

mrmf_status mrmf_batch_autotune(mrmf_batch b, const void* d_ws, const float* d_theta_all, const void* d_X,
                                void* d_Y, mrmf_stream stream, int32_t* out) {
    mrmf_status st = check_call(b, d_ws, d_theta_all, d_X, d_Y);
    if (st != MRMF_OK) return st;
    if (!out) return MRMF_E_INVALID_ARG;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return MRMF_E_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return MRMF_E_HIP;
    }
    float best = 0.f;
    int best_i = -1;
    const int32_t R0 = b->rc, B0 = b->block, S0 = b->sched;
    // candidates: every shape with the runs schedule, then with the windows schedule, then per-XCD chunks
    for (int i = 0; i < 3 * mrmf::kNumShapes && st == MRMF_OK; ++i) {
        b->rc = mrmf::kShapes[i % mrmf::kNumShapes].rc;
        b->block = mrmf::kShapes[i % mrmf::kNumShapes].block;
        b->sched = i / mrmf::kNumShapes;
        if (b->block > mrmf::kBatchTileWords / b->nvec) continue;
        st = launch(b, d_ws, d_theta_all, d_X, d_Y, s);  // warm-up
        if (st != MRMF_OK) break;
        hipEventRecord(e0, s);
        for (int r = 0; r < 3 && st == MRMF_OK; ++r) st = launch(b, d_ws, d_theta_all, d_X, d_Y, s);
        hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) st = MRMF_E_HIP;
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        if (st == MRMF_OK && (best_i < 0 || ms < best)) {
            best = ms;
            best_i = i;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (best_i < 0) {
        b->rc = R0;
        b->block = B0;
        b->sched = S0;
        return st != MRMF_OK ? st : MRMF_E_HIP;
    }
    b->rc = mrmf::kShapes[best_i % mrmf::kNumShapes].rc;
    b->block = mrmf::kShapes[best_i % mrmf::kNumShapes].block;
    b->sched = best_i / mrmf::kNumShapes;
    out[0] = mrmf::rmax_of(b->rc, b->nvec);
    out[1] = b->block;
    out[2] = best_i;
    return st;
}

}  // extern "C"
