// Runs an emulated kernel `mrmf_spec(theta, x, y, skip)` (compiled from generated HIP source together
// with hip_emu.h) over a grid of blocks on host threads.  Test infrastructure only.
#include <pthread.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "hip_emu.h"

thread_local emu_dim3 threadIdx, blockIdx;
emu_dim3 gridDim, blockDim;
double emu_shfl_slot[16][64];
unsigned long long emu_ballot_slot[16][64];
int emu_dpp_slot[16][64];

void emu_dpp_unsupported(int ctrl) {
    std::fprintf(stderr, "emu: DPP control 0x%x is not emulated\n", ctrl);
    std::fflush(stderr);
    std::abort();
}

void emu_uniform_failed(long long mine, long long first) {
    std::fprintf(stderr, "emu: readfirstlane of a non-uniform value (lane %u has %lld, lane 0 %lld)\n", threadIdx.x,
                 mine, first);
    std::fflush(stderr);
    std::abort();
}

namespace {
pthread_barrier_t g_block_bar;
pthread_barrier_t g_wave_bar[16];
struct Buf {
    const char* p;
    size_t n;
    const char* name;
};
std::vector<Buf> g_bufs;
Buf g_extra{nullptr, 0, ""};  // one more buffer of the next launch (the adjoint kernel's partial sums)
int g_fault = 0;
}  // namespace

void emu_syncthreads() { pthread_barrier_wait(&g_block_bar); }
void emu_wave_barrier() { pthread_barrier_wait(&g_wave_bar[threadIdx.x >> 6]); }

void emu_check(const void* p, size_t n, const char* what) {
    const char* c = static_cast<const char*>(p);
    for (const Buf& b : g_bufs)
        if (c >= b.p && c + n <= b.p + b.n) return;
    std::fprintf(stderr, "emu: %s of %zu bytes at %p outside every buffer (block %u thread %u)\n", what, n, p,
                 blockIdx.x, threadIdx.x);
    for (const Buf& b : g_bufs) std::fprintf(stderr, "  %s: [%p, %p)\n", b.name, (const void*)b.p, (const void*)(b.p + b.n));
    std::fflush(stderr);
    std::abort();
}

// A generated source defines one of the kernels: the plain matvec, the Chebyshev-step form, or the
// adjoint's coupling-gradient kernel.
extern "C" void mrmf_spec(const void* theta, const void* x, void* y, const int* skip) __attribute__((weak));
extern "C" void mrmf_grad(const double* theta, const void* x, const void* g, void* gx, double* partial)
    __attribute__((weak));
extern "C" void mrmf_sector(const void* theta, const void* x, void* y, const int* skip, const void* lab)
    __attribute__((weak));
extern "C" void mrmf_spec_cheb(const void* theta, const void* x, void* y, void* acc, double ea, double eb, double eg,
                               double ecr, double eci, const int* skip) __attribute__((weak));
extern "C" void mrmf_sector_cheb(const void* theta, const void* x, void* y, void* acc, double ea, double eb, double eg,
                                 double ecr, double eci, const int* skip, const void* lab) __attribute__((weak));

namespace {
struct Arg {
    unsigned tid, b0, b1;
    const void *theta, *x;
    void* y;
};
// Chebyshev-step launch: accumulator and epilogue scalars (cheb = false: the plain matvec)
struct ChebCall {
    bool cheb = false;
    void* acc = nullptr;
    double ea = 0, eb = 0, eg = 0, ecr = 0, eci = 0;
} g_cheb;
// Adjoint-kernel launch: its extra pointers (the launch's `theta`, `x`, `y` slots hold theta, x, gx)
struct GradCall {
    bool on = false;
    const void* g = nullptr;
    double* partial = nullptr;
} g_grad;
bool g_sector = false;        // the launch runs the generated sector kernel
const void* g_lab = nullptr;  // its packed-digit table
// One host thread per GPU thread of the block, kept for every block of the range; a block barrier
// separates consecutive blocks (their __shared__ storage is the same static storage).
void* thread_main(void* a) {
    Arg* g = static_cast<Arg*>(a);
    threadIdx = emu_dim3{g->tid, 0, 0};
    for (unsigned b = g->b0; b < g->b1; ++b) {
        blockIdx = emu_dim3{b, 0, 0};
        if (g_sector && g_cheb.cheb)
            mrmf_sector_cheb(g->theta, g->x, g->y, g_cheb.acc, g_cheb.ea, g_cheb.eb, g_cheb.eg, g_cheb.ecr, g_cheb.eci,
                             nullptr, g_lab);
        else if (g_sector)
            mrmf_sector(g->theta, g->x, g->y, nullptr, g_lab);
        else if (g_grad.on)
            mrmf_grad(static_cast<const double*>(g->theta), g->x, g_grad.g, g->y, g_grad.partial);
        else if (g_cheb.cheb)
            mrmf_spec_cheb(g->theta, g->x, g->y, g_cheb.acc, g_cheb.ea, g_cheb.eb, g_cheb.eg, g_cheb.ecr, g_cheb.eci,
                           nullptr);
        else
            mrmf_spec(g->theta, g->x, g->y, nullptr);
        pthread_barrier_wait(&g_block_bar);
    }
    return nullptr;
}
}  // namespace

// Runs blocks [b0, b1) of a grid of `grid` blocks (b1 = 0: all of them).
extern "C" int emu_run_range(unsigned grid, unsigned block, const void* theta, size_t theta_bytes, const void* x,
                             size_t x_bytes, void* y, size_t y_bytes, unsigned b0, unsigned b1);

extern "C" int emu_run(unsigned grid, unsigned block, const void* theta, size_t theta_bytes, const void* x,
                       size_t x_bytes, void* y, size_t y_bytes) {
    return emu_run_range(grid, block, theta, theta_bytes, x, x_bytes, y, y_bytes, 0, 0);
}

extern "C" int emu_run_range(unsigned grid, unsigned block, const void* theta, size_t theta_bytes, const void* x,
                             size_t x_bytes, void* y, size_t y_bytes, unsigned b0, unsigned b1) {
    if (b1 == 0 || b1 > grid) b1 = grid;
    if (block == 0 || block % 64 != 0 || block > 1024) return -1;
    if (g_sector ? (g_cheb.cheb ? mrmf_sector_cheb == nullptr : mrmf_sector == nullptr)
                 : g_grad.on ? mrmf_grad == nullptr : g_cheb.cheb ? mrmf_spec_cheb == nullptr : mrmf_spec == nullptr)
        return -3;
    g_bufs = {{static_cast<const char*>(x), x_bytes, "x"}, {static_cast<const char*>(y), y_bytes, "y"},
              {static_cast<const char*>(theta), theta_bytes, "theta"}};
    if (g_cheb.cheb) g_bufs.push_back({static_cast<const char*>(g_cheb.acc), x_bytes, "acc"});
    if (g_grad.on) g_bufs.push_back({static_cast<const char*>(g_grad.g), x_bytes, "g"});
    if (g_extra.p) g_bufs.push_back(g_extra);
    gridDim = emu_dim3{grid, 1, 1};
    blockDim = emu_dim3{block, 1, 1};
    const unsigned nw = block / 64;
    pthread_barrier_init(&g_block_bar, nullptr, block);
    for (unsigned w = 0; w < nw; ++w) pthread_barrier_init(&g_wave_bar[w], nullptr, 64);
    std::vector<pthread_t> th(block);
    std::vector<Arg> args(block);
    pthread_attr_t attr;
    pthread_attr_init(&attr);
    pthread_attr_setstacksize(&attr, 1 << 20);
    int rc = 0;
    unsigned started = 0;
    for (unsigned t = 0; t < block; ++t) {
        args[t] = Arg{t, b0, b1, theta, x, y};
        if (pthread_create(&th[t], &attr, thread_main, &args[t]) != 0) {
            rc = -2;
            break;
        }
        ++started;
    }
    if (rc != 0) {  // cannot run a partial block: report and stop (the started threads wait at a barrier)
        std::fprintf(stderr, "emu: could not start %u threads\n", block);
        std::abort();
    }
    for (unsigned t = 0; t < started; ++t) pthread_join(th[t], nullptr);
    pthread_attr_destroy(&attr);
    pthread_barrier_destroy(&g_block_bar);
    for (unsigned w = 0; w < nw; ++w) pthread_barrier_destroy(&g_wave_bar[w]);
    return g_fault;
}

// The Chebyshev-step kernel over blocks [b0, b1): y (prev) and acc are updated in place; acc has the
// length of x.
extern "C" int emu_run_cheb(unsigned grid, unsigned block, const void* theta, size_t theta_bytes, const void* x,
                            size_t x_bytes, void* prev, void* acc, double ea, double eb, double eg, double ecr,
                            double eci, unsigned b0, unsigned b1) {
    g_cheb = ChebCall{true, acc, ea, eb, eg, ecr, eci};
    const int rc = emu_run_range(grid, block, theta, theta_bytes, x, x_bytes, prev, x_bytes, b0, b1);
    g_cheb = ChebCall{};
    return rc;
}

// The adjoint kernel over all `grid` blocks of 256 threads: gx (length of x) = H g, partial holds
// grid x n_params doubles (a buffer of its own: registered through g_bufs below).
extern "C" int emu_run_grad(unsigned grid, const void* theta, size_t theta_bytes, const void* x, size_t x_bytes,
                            const void* g, void* gx, void* partial, size_t partial_bytes) {
    g_grad = GradCall{true, g, static_cast<double*>(partial)};
    g_extra = {static_cast<const char*>(partial), partial_bytes, "partial"};
    const int rc = emu_run_range(grid, 256, theta, theta_bytes, x, x_bytes, gx, x_bytes, 0, 0);
    g_grad = GradCall{};
    g_extra = {nullptr, 0, ""};
    return rc;
}

// The generated sector kernel over all `grid` blocks of 256 threads (packed vectors x, y; lab: the packed
// digits of every state, lab_bytes bytes).
extern "C" int emu_run_sector(unsigned grid, const void* theta, size_t theta_bytes, const void* x, size_t x_bytes,
                              void* y, size_t y_bytes, const void* lab, size_t lab_bytes) {
    g_sector = true;
    g_lab = lab;
    g_extra = {static_cast<const char*>(lab), lab_bytes, "lab"};
    const int rc = emu_run_range(grid, 256, theta, theta_bytes, x, x_bytes, y, y_bytes, 0, 0);
    g_sector = false;
    g_lab = nullptr;
    g_extra = {nullptr, 0, ""};
    return rc;
}

// The sector kernel with the Chebyshev-step epilogue over all `grid` blocks of 256 threads: prev and acc
// (packed vectors, the length of x) are updated in place.
extern "C" int emu_run_sector_cheb(unsigned grid, const void* theta, size_t theta_bytes, const void* x, size_t x_bytes,
                                   void* prev, void* acc, double ea, double eb, double eg, double ecr, double eci,
                                   const void* lab, size_t lab_bytes) {
    g_sector = true;
    g_lab = lab;
    g_extra = {static_cast<const char*>(lab), lab_bytes, "lab"};
    g_cheb = ChebCall{true, acc, ea, eb, eg, ecr, eci};
    const int rc = emu_run_range(grid, 256, theta, theta_bytes, x, x_bytes, prev, x_bytes, 0, 0);
    g_cheb = ChebCall{};
    g_sector = false;
    g_lab = nullptr;
    g_extra = {nullptr, 0, ""};
    return rc;
}
