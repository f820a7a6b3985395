// Host emulation of the small HIP device subset used by the generated matvec kernels, so that a
// generated kernel can be compiled for x86 and run on the CPU with every memory access checked.
//
// Test infrastructure only.  Each GPU thread of a block is a host thread; __syncthreads is a barrier
// over the block, __shfl_down exchanges through a per-wave buffer between two wave barriers.  Blocks
// run one after another, so __shared__ (mapped to function-local static storage) is private to the
// running block.  Buffer loads and stores follow the raw-buffer rule the kernels rely on: an access
// whose VGPR offset is at or beyond the record count reads 0 / writes nothing; any other access must
// fall inside a buffer registered with emu_register, or the process aborts with a message.
#pragma once

#include <pthread.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#define __global__
#define __device__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __constant__ static const
using std::fma;

struct emu_dim3 {
    unsigned x, y, z;
};
extern thread_local emu_dim3 threadIdx, blockIdx;
extern emu_dim3 gridDim, blockDim;

void emu_syncthreads();
void emu_wave_barrier();
extern double emu_shfl_slot[16][64];
#define __syncthreads() emu_syncthreads()

template <typename T>
inline T __shfl_down(T v, int k, int width) {
    (void)width;
    const unsigned t = threadIdx.x, w = t >> 6, l = t & 63u;
    emu_shfl_slot[w][l] = static_cast<double>(v);
    emu_wave_barrier();
    const T r = (l + k < 64u) ? static_cast<T>(emu_shfl_slot[w][l + k]) : v;
    emu_wave_barrier();
    return r;
}

extern unsigned long long emu_ballot_slot[16][64];
inline unsigned long long __ballot(int pred) {
    const unsigned t = threadIdx.x, w = t >> 6, l = t & 63u;
    emu_ballot_slot[w][l] = pred ? 1ull : 0ull;
    emu_wave_barrier();
    unsigned long long m = 0;
    for (unsigned k = 0; k < 64; ++k) m |= emu_ballot_slot[w][k] << k;
    emu_wave_barrier();
    return m;
}
inline int __popcll(unsigned long long v) { return __builtin_popcountll(v); }
// every lane must hold the same value where the kernels use this: the emulation checks it
void emu_uniform_failed(long long mine, long long first);
inline int emu_readfirstlane(int v) {
    const unsigned t = threadIdx.x, w = t >> 6, l = t & 63u;
    emu_ballot_slot[w][l] = static_cast<unsigned long long>(static_cast<unsigned>(v));
    emu_wave_barrier();
    const int first = static_cast<int>(static_cast<unsigned>(emu_ballot_slot[w][0]));
    emu_wave_barrier();
    if (first != v) emu_uniform_failed(v, first);
    return first;
}
#define __builtin_amdgcn_readfirstlane(v) emu_readfirstlane((int)(v))

// DPP lane moves (the controls the kernels use: quad_perm, row_mirror, row_half_mirror, row_bcast:15,
// row_bcast:31).  A lane of a row or bank outside the masks keeps `old`; a lane with no source lane
// keeps `old` unless bound_ctrl, then 0.
extern int emu_dpp_slot[16][64];
void emu_dpp_unsupported(int ctrl);
inline int emu_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl) {
    const unsigned t = threadIdx.x, w = t >> 6, l = t & 63u, row = l >> 4;
    emu_dpp_slot[w][l] = src;
    emu_wave_barrier();
    int s = -1;
    if (ctrl >= 0 && ctrl <= 0xff) s = static_cast<int>((l & ~3u) + ((static_cast<unsigned>(ctrl) >> (2 * (l & 3u))) & 3u));
    else if (ctrl == 0x140) s = static_cast<int>((row << 4) + (15u - (l & 15u)));
    else if (ctrl == 0x141) s = static_cast<int>((l & ~7u) + (7u - (l & 7u)));
    else if (ctrl == 0x142) s = row >= 1 ? static_cast<int>(row << 4) - 1 : -1;
    else if (ctrl == 0x143) s = row >= 2 ? 31 : -1;
    else emu_dpp_unsupported(ctrl);
    int r = old;
    if (((row_mask >> row) & 1) && ((bank_mask >> ((l >> 2) & 3u)) & 1)) {
        if (s >= 0) r = emu_dpp_slot[w][s];
        else if (bound_ctrl) r = 0;
    }
    emu_wave_barrier();
    return r;
}
#define __builtin_amdgcn_update_dpp(old, src, ctrl, row_mask, bank_mask, bound) \
    emu_update_dpp((old), (src), (ctrl), (row_mask), (bank_mask), (bound))
#define __builtin_amdgcn_sched_barrier(mask) ((void)0)  /* instruction scheduling only */
#define MRMF_GROUP_FENCE(a, b) ((void)0)                 /* orders the generated code only */

inline unsigned long long __umul64hi(unsigned long long a, unsigned long long b) {
    return static_cast<unsigned long long>((static_cast<unsigned __int128>(a) * b) >> 64);
}

struct emu_rsrc {
    const char* base;
    uint32_t num;
};
#define __amdgpu_buffer_rsrc_t emu_rsrc
#define __builtin_amdgcn_make_buffer_rsrc(p, stride, num, flags) emu_rsrc{(const char*)(p), (uint32_t)(num)}

void emu_check(const void* p, size_t n, const char* what);

typedef unsigned emu_u2 __attribute__((ext_vector_type(2)));
typedef unsigned emu_u4 __attribute__((ext_vector_type(4)));

template <typename V>
inline V emu_load(emu_rsrc r, int vo, int so) {
    V v;
    if (static_cast<uint32_t>(vo) >= r.num) {
        std::memset(&v, 0, sizeof v);
        return v;
    }
    const char* p = r.base + static_cast<uint32_t>(vo) + static_cast<uint32_t>(so);
    emu_check(p, sizeof v, "buffer load");
    std::memcpy(&v, p, sizeof v);
    return v;
}

template <typename V>
inline void emu_store(V v, emu_rsrc r, int vo, int so) {
    if (static_cast<uint32_t>(vo) >= r.num) return;
    char* p = const_cast<char*>(r.base) + static_cast<uint32_t>(vo) + static_cast<uint32_t>(so);
    emu_check(p, sizeof v, "buffer store");
    std::memcpy(p, &v, sizeof v);
}

#define __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, aux) emu_load<emu_u4>((r), (vo), (so))
#define __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, aux) emu_load<unsigned>((r), (vo), (so))
#define __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, aux) emu_load<emu_u2>((r), (vo), (so))
#define __builtin_amdgcn_raw_buffer_store_b128(v, r, vo, so, aux) emu_store<emu_u4>((v), (r), (vo), (so))
#define __builtin_amdgcn_raw_buffer_store_b64(v, r, vo, so, aux) emu_store<emu_u2>((v), (r), (vo), (so))
