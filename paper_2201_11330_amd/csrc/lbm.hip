// liblbm.so: host runtime and C interface (include/lbm.h) of the gfx950 LBM
// time step.  Validates arguments, owns the context, picks the kernel
// instantiation (lattice x storage x walls x force) and launches it on the
// caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "../../include/lbm.h"
#include "adjoint.hpp"
#include "kernels.hpp"

using namespace imexlbm;

namespace {

thread_local char g_last_error[512] = "";

lbm_status fail(lbm_status st, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return st;
}

lbm_status hip_fail(hipError_t e, const char* what)
{
    return fail(LBM_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define LBM_HIP(call)                                      \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return hip_fail(e_, #call);  \
    } while (0)

size_t storage_size(lbm_storage s)
{
    switch (s) {
    case LBM_F64: return 8;
    case LBM_F32: return 4;
    case LBM_F16_DEV:
    case LBM_BF16_DEV: return 2;
    }
    return 0;
}

// Steps per captured graph (even, so a replay returns the two-lattice
// buffers and the AA parity to where they started).
constexpr int kGraphSteps = 32;

// Non-temporal stores (and unshared loads) in the step kernels.
constexpr bool kNtStores = true;

// Tile length of the stored state: 4096 nodes (the fastest of 256..8192
// measured on MI355X for D3Q19 FP64 and FP16), or N rounded up to a power of
// two for smaller boxes.
int tile_shift(unsigned long long N)
{
    int s = 0;
    while (s < 12 && (1ull << s) < N) ++s;
    return s;
}

}  // namespace

struct lbm_ctx {
    lbm_lattice lattice;
    int D, Q;
    int nx, ny, nz;
    unsigned N;
    int S;     // log2 of the tile length of the stored state
    size_t state_elems;  // elements of one stored state (whole tiles)
    double tau, omega;
    double F[3];
    int bc[3];
    lbm_storage storage;
    unsigned flags;
    bool walls, force, aa;

    bool bound = false;
    void* buf[2] = {nullptr, nullptr};
    int cur = 0;  // AB: buffer holding the current state
    hipStream_t stream = nullptr;
    bool state_valid = false;
    long long steps = 0;

    unsigned* links = nullptr;     // per-node link bits of a solid mask (lbm_set_solid)
    double* d_partials = nullptr;  // kReduceBlocks * 5 + 4 doubles
    double* h_result = nullptr;    // 4 doubles, pinned

    int bx_shift = 8;
    dim3 grid, block;

    // LBM_FLAG_GRAPH: kGraphSteps steps captured once, replayed by lbm_step.
    bool use_graph = false;
    hipStream_t capture_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
};

namespace {

void plan_launch(lbm_ctx* c)
{
    int bx = 1, shift = 0;
    while (bx < c->nx && bx < 256) {
        bx <<= 1;
        ++shift;
    }
    const int by = 256 / bx;
    c->bx_shift = shift;
    c->block = dim3(256, 1, 1);
    c->grid = dim3((c->nx + bx - 1) / bx, (c->ny + by - 1) / by, c->nz);
}

Dims dims_of(const lbm_ctx* c)
{
    Dims g;
    g.nx = c->nx;
    g.ny = c->ny;
    g.nz = c->nz;
    for (int d = 0; d < 3; ++d) g.bc[d] = c->bc[d];
    g.N = c->N;
    g.S = c->S;
    g.links = c->links;
    return g;
}

// The gather mode of the current state (AA parity after an odd number of
// steps means the next step is odd).
int state_mode(const lbm_ctx* c)
{
    if (!c->aa) return kPull;
    return (c->steps & 1) ? kPullFlip : kLocal;
}

IoArgs io_args(const lbm_ctx* c)
{
    IoArgs p;
    p.g = dims_of(c);
    p.bx_shift = c->bx_shift;
    p.mode = state_mode(c);
    for (int d = 0; d < 3; ++d) p.F[d] = c->F[d];
    return p;
}

template <class C>
StepArgs<C> step_args(const lbm_ctx* c)
{
    StepArgs<C> p;
    p.g = dims_of(c);
    p.bx_shift = c->bx_shift;
    p.c.omega = C(c->omega);
    for (int d = 0; d < 3; ++d) p.c.F[d] = C(c->F[d]);
    const double half = 1.0 - 0.5 * c->omega;
    p.c.k3 = C(3.0 * half);
    p.c.k9 = C(9.0 * half);
    return p;
}

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// Byte offsets inside the lbm_adjoint workspace.
struct WorkspaceLayout {
    size_t state_bytes;  // one stored state (also the checkpoint stride)
    size_t seg, lam0, lam1, acc, result, total;
    size_t nblocks, acc_doubles;
};

WorkspaceLayout workspace_layout(const lbm_ctx* c, int k);

// Kernel instantiations of one lattice and storage.
template <int L, class S>
struct Impl {
    template <bool W, bool F>
    static void step_ab(lbm_ctx* c, const S* src, S* dst)
    {
        hipLaunchKernelGGL((k_step_ab<L, S, W, F, kNtStores>), c->grid, c->block, 0, c->stream, src, dst,
                           step_args<typename Store<S>::C>(c));
    }
    template <bool W, bool F>
    static void step_aa(lbm_ctx* c, S* A, bool odd)
    {
        if (odd)
            hipLaunchKernelGGL((k_step_aa_odd<L, S, W, F, kNtStores>), c->grid, c->block, 0, c->stream, A,
                               step_args<typename Store<S>::C>(c));
        else
            hipLaunchKernelGGL((k_step_aa_even<L, S, W, F, kNtStores>), c->grid, c->block, 0, c->stream, A,
                               step_args<typename Store<S>::C>(c));
    }

    // Captures kGraphSteps steps starting from an even step count (buffer 0
    // current, AA even parity) on a private stream; the context's launch
    // stream and counters are restored afterwards.
    static lbm_status capture(lbm_ctx* c)
    {
        if (!c->capture_stream) LBM_HIP(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
        hipError_t e = hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        hipStream_t saved_stream = c->stream;
        const int saved_cur = c->cur;
        const long long saved_steps = c->steps;
        c->stream = c->capture_stream;
        c->cur = 0;
        c->steps = 0;
        const lbm_status st = eager(c, kGraphSteps);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(c->capture_stream, &g);
        c->stream = saved_stream;
        c->cur = saved_cur;
        c->steps = saved_steps;
        if (st != LBM_OK || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return st != LBM_OK ? st : hip_fail(e, "hipStreamEndCapture");
        }
        c->graph = g;
        e = hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(c->graph);
            c->graph = nullptr;
            c->graph_exec = nullptr;
            return hip_fail(e, "hipGraphInstantiate");
        }
        return LBM_OK;
    }

    static lbm_status step(lbm_ctx* c, int n)
    {
        if (!c->use_graph || n < kGraphSteps) return eager(c, n);
        if (c->steps & 1) {  // align to the captured parity
            lbm_status st = eager(c, 1);
            if (st) return st;
            --n;
        }
        if (!c->graph_exec) {
            lbm_status st = capture(c);
            if (st) return st;
        }
        for (; n >= kGraphSteps; n -= kGraphSteps) {
            LBM_HIP(hipGraphLaunch(c->graph_exec, c->stream));
            c->steps += kGraphSteps;
        }
        return eager(c, n);
    }

    static lbm_status eager(lbm_ctx* c, int n)
    {
        for (int i = 0; i < n; ++i) {
            if (c->aa) {
                S* A = static_cast<S*>(c->buf[0]);
                const bool odd = c->steps & 1;
                if (c->walls)
                    c->force ? step_aa<true, true>(c, A, odd) : step_aa<true, false>(c, A, odd);
                else
                    c->force ? step_aa<false, true>(c, A, odd) : step_aa<false, false>(c, A, odd);
            } else {
                const S* src = static_cast<const S*>(c->buf[c->cur]);
                S* dst = static_cast<S*>(c->buf[1 - c->cur]);
                if (c->walls)
                    c->force ? step_ab<true, true>(c, src, dst) : step_ab<true, false>(c, src, dst);
                else
                    c->force ? step_ab<false, true>(c, src, dst) : step_ab<false, false>(c, src, dst);
                c->cur = 1 - c->cur;
            }
            ++c->steps;
        }
        LBM_HIP(hipGetLastError());
        return LBM_OK;
    }

    // One two-lattice step between explicit buffers.
    static void step_between(lbm_ctx* c, const S* src, S* dst)
    {
        if (c->walls)
            c->force ? step_ab<true, true>(c, src, dst) : step_ab<true, false>(c, src, dst);
        else
            c->force ? step_ab<false, true>(c, src, dst) : step_ab<false, false>(c, src, dst);
    }

    using C = typename Store<S>::C;

    static AdjArgs<C> adj_args(const lbm_ctx* c)
    {
        AdjArgs<C> p;
        p.g = dims_of(c);
        p.bx_shift = c->bx_shift;
        p.omega = C(c->omega);
        for (int d = 0; d < 3; ++d) p.F[d] = C(c->F[d]);
        p.half = C(1.0 - 0.5 * c->omega);
        return p;
    }

    template <bool W, bool F>
    static void adj_step(lbm_ctx* c, const S* g, const C* lin, C* lout, double* acc)
    {
        hipLaunchKernelGGL((k_adjoint_step<L, S, W, F>), c->grid, c->block, 0, c->stream, g, lin, lout,
                           acc, adj_args(c));
    }

    // Backward sweep over n steps with checkpoints every k steps; see
    // lbm_adjoint.  ws holds (k-1) state buffers, two lambda fields and the
    // per-workgroup accumulators.
    static lbm_status adjoint(lbm_ctx* c, int n, int k, const void* ckpt, void* ws,
                              const double* u0, const double* ubar, double* u0bar, double* out4)
    {
        const WorkspaceLayout W = workspace_layout(c, k);
        char* w = static_cast<char*>(ws);
        C* lam[2] = {reinterpret_cast<C*>(w + W.lam0), reinterpret_cast<C*>(w + W.lam1)};
        double* acc = reinterpret_cast<double*>(w + W.acc);
        double* result = reinterpret_cast<double*>(w + W.result);
        const Dims g = dims_of(c);
        hipLaunchKernelGGL(k_fill_zero, dim3((W.acc_doubles + 255) / 256), dim3(256), 0, c->stream, acc,
                           W.acc_doubles);
        if (c->walls)
            hipLaunchKernelGGL((k_adjoint_seed<L, S, true>), c->grid, c->block, 0, c->stream, ubar, lam[0],
                               acc, g, c->bx_shift);
        else
            hipLaunchKernelGGL((k_adjoint_seed<L, S, false>), c->grid, c->block, 0, c->stream, ubar, lam[0],
                               acc, g, c->bx_shift);
        int cur = 0;
        const char* ck = static_cast<const char*>(ckpt);
        for (int s = n / k - 1; s >= 0; --s) {
            const S* state0 = reinterpret_cast<const S*>(ck + size_t(s) * W.state_bytes);
            auto state = [&](int j) -> const S* {
                return j == 0 ? state0 : reinterpret_cast<const S*>(w + W.seg + size_t(j - 1) * W.state_bytes);
            };
            for (int j = 1; j < k; ++j)
                step_between(c, state(j - 1), const_cast<S*>(state(j)));
            for (int j = k - 1; j >= 0; --j) {
                if (c->walls)
                    c->force ? adj_step<true, true>(c, state(j), lam[cur], lam[1 - cur], acc)
                             : adj_step<true, false>(c, state(j), lam[cur], lam[1 - cur], acc);
                else
                    c->force ? adj_step<false, true>(c, state(j), lam[cur], lam[1 - cur], acc)
                             : adj_step<false, false>(c, state(j), lam[cur], lam[1 - cur], acc);
                cur = 1 - cur;
            }
        }
        if (c->walls)
            hipLaunchKernelGGL((k_adjoint_init_map<L, S, true>), c->grid, c->block, 0, c->stream, lam[cur], u0,
                               u0bar, g, c->bx_shift);
        else
            hipLaunchKernelGGL((k_adjoint_init_map<L, S, false>), c->grid, c->block, 0, c->stream, lam[cur], u0,
                               u0bar, g, c->bx_shift);
        hipLaunchKernelGGL(k_adjoint_sum, dim3(1), dim3(256), 0, c->stream, acc, W.nblocks, result);
        LBM_HIP(hipGetLastError());
        LBM_HIP(hipMemcpyAsync(out4, result, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        LBM_HIP(hipStreamSynchronize(c->stream));
        return LBM_OK;
    }

    static lbm_status build_links(lbm_ctx* c, const unsigned char* mask)
    {
        Dims g = dims_of(c);
        g.links = nullptr;
        hipLaunchKernelGGL((k_build_links<L>), c->grid, c->block, 0, c->stream, mask, c->links, g,
                           c->bx_shift);
        LBM_HIP(hipGetLastError());
        return LBM_OK;
    }

    static lbm_status wall_force(lbm_ctx* c)
    {
        IoArgs p = io_args(c);
        const S* A = static_cast<const S*>(c->buf[c->cur]);
        hipLaunchKernelGGL((k_wall_force<L, S>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, c->stream,
                           A, c->d_partials, p);
        hipLaunchKernelGGL(k_sum3, dim3(1), dim3(kReduceThreads), 0, c->stream, c->d_partials,
                           kReduceBlocks, c->d_partials + 5 * size_t(kReduceBlocks));
        LBM_HIP(hipGetLastError());
        return LBM_OK;
    }

    static lbm_status import(lbm_ctx* c, const double* f, const double* rho, const double* u,
                             const double* noise)
    {
        IoArgs p = io_args(c);
        S* A = static_cast<S*>(c->buf[c->cur]);
        if (c->walls)
            hipLaunchKernelGGL((k_import<L, S, true>), c->grid, c->block, 0, c->stream, A, f, rho, u,
                               noise, p);
        else
            hipLaunchKernelGGL((k_import<L, S, false>), c->grid, c->block, 0, c->stream, A, f, rho, u,
                               noise, p);
        LBM_HIP(hipGetLastError());
        return LBM_OK;
    }

    static lbm_status export_f(lbm_ctx* c, double* f)
    {
        IoArgs p = io_args(c);
        const S* A = static_cast<const S*>(c->buf[c->cur]);
        if (c->walls)
            hipLaunchKernelGGL((k_export<L, S, true>), c->grid, c->block, 0, c->stream, A, f, p);
        else
            hipLaunchKernelGGL((k_export<L, S, false>), c->grid, c->block, 0, c->stream, A, f, p);
        LBM_HIP(hipGetLastError());
        return LBM_OK;
    }

    template <class O>
    static void moments_t(lbm_ctx* c, O* rho, O* u)
    {
        IoArgs p = io_args(c);
        const S* A = static_cast<const S*>(c->buf[c->cur]);
        if (c->walls)
            hipLaunchKernelGGL((k_moments<L, S, true, O>), c->grid, c->block, 0, c->stream, A, rho, u,
                               p);
        else
            hipLaunchKernelGGL((k_moments<L, S, false, O>), c->grid, c->block, 0, c->stream, A, rho,
                               u, p);
    }

    static lbm_status moments(lbm_ctx* c, void* rho, void* u, int f32)
    {
        if (f32)
            moments_t<float>(c, static_cast<float*>(rho), static_cast<float*>(u));
        else
            moments_t<double>(c, static_cast<double*>(rho), static_cast<double*>(u));
        LBM_HIP(hipGetLastError());
        return LBM_OK;
    }

    static lbm_status reduce(lbm_ctx* c)
    {
        IoArgs p = io_args(c);
        const S* A = static_cast<const S*>(c->buf[c->cur]);
        if (c->walls)
            hipLaunchKernelGGL((k_reduce_partials<L, S, true>), dim3(kReduceBlocks),
                               dim3(kReduceThreads), 0, c->stream, A, c->d_partials, p);
        else
            hipLaunchKernelGGL((k_reduce_partials<L, S, false>), dim3(kReduceBlocks),
                               dim3(kReduceThreads), 0, c->stream, A, c->d_partials, p);
        hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kReduceThreads), 0, c->stream, c->d_partials,
                           kReduceBlocks, int(Store<S>::kDeviation),
                           c->d_partials + 5 * size_t(kReduceBlocks));
        LBM_HIP(hipGetLastError());
        return LBM_OK;
    }
};

// Calls Impl<L, S>::fn(c, args...) for the context's lattice and storage.
#define LBM_DISPATCH_STORAGE(c, LK, CALL)                                            \
    switch ((c)->storage) {                                                          \
    case LBM_F64: { using I = Impl<LK, double>; return I::CALL; }                    \
    case LBM_F32: { using I = Impl<LK, float>; return I::CALL; }                     \
    case LBM_F16_DEV: { using I = Impl<LK, __half>; return I::CALL; }                \
    case LBM_BF16_DEV: { using I = Impl<LK, __hip_bfloat16>; return I::CALL; }       \
    }
#define LBM_DISPATCH(c, CALL)                                                        \
    do {                                                                             \
        switch ((c)->lattice) {                                                      \
        case LBM_D2Q9: LBM_DISPATCH_STORAGE(c, 0, CALL) break;                       \
        case LBM_D3Q19: LBM_DISPATCH_STORAGE(c, 1, CALL) break;                      \
        case LBM_D3Q27: LBM_DISPATCH_STORAGE(c, 2, CALL) break;                      \
        }                                                                            \
        return fail(LBM_EINVAL, "unknown lattice/storage");                          \
    } while (0)

lbm_status need_bound(const lbm_ctx* c)
{
    if (!c) return fail(LBM_EINVAL, "null context");
    if (!c->bound) return fail(LBM_ENOTBOUND, "context has no buffers bound (lbm_bind)");
    return LBM_OK;
}

lbm_status need_state(const lbm_ctx* c)
{
    lbm_status st = need_bound(c);
    if (st) return st;
    if (!c->state_valid)
        return fail(LBM_ESTATE, "populations not initialised (lbm_init_equilibrium / lbm_set_populations)");
    return LBM_OK;
}

lbm_status check_device_ptr(const void* p, const char* name, bool allow_null)
{
    if (!p) return allow_null ? LBM_OK : fail(LBM_EINVAL, "%s is NULL", name);
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(LBM_EINVAL, "%s is not a HIP allocation", name);
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
        return fail(LBM_EINVAL, "%s is not device memory", name);
    int dev = -1;
    LBM_HIP(hipGetDevice(&dev));
    if (attr.device != dev) return fail(LBM_EINVAL, "%s is on device %d, current is %d", name, attr.device, dev);
    return LBM_OK;
}

WorkspaceLayout workspace_layout(const lbm_ctx* c, int k)
{
    WorkspaceLayout L;
    const size_t elem = storage_size(c->storage);
    const size_t celem = c->storage == LBM_F64 ? 8 : 4;  // arithmetic type of lambda
    L.state_bytes = round256(c->state_elems * elem);
    L.nblocks = size_t(c->grid.x) * c->grid.y * c->grid.z;
    L.acc_doubles = L.nblocks * kAccSlots;
    L.seg = 0;
    L.lam0 = L.seg + size_t(k > 1 ? k - 1 : 0) * L.state_bytes;
    L.lam1 = L.lam0 + round256(c->state_elems * celem);
    L.acc = L.lam1 + round256(c->state_elems * celem);
    L.result = L.acc + round256(L.acc_doubles * sizeof(double));
    L.total = L.result + 256;
    return L;
}

lbm_status adjoint_any(lbm_ctx* c, int n, int k, const void* ckpt, void* ws, const double* u0,
                       const double* ubar, double* u0bar, double* out4)
{
    LBM_DISPATCH(c, adjoint(c, n, k, ckpt, ws, u0, ubar, u0bar, out4));
}

lbm_status import_any(lbm_ctx* c, const double* f, const double* rho, const double* u,
                      const double* noise)
{
    LBM_DISPATCH(c, import(c, f, rho, u, noise));
}

lbm_status reduce_launch(lbm_ctx* c)
{
    LBM_DISPATCH(c, reduce(c));
}

lbm_status build_links_any(lbm_ctx* c, const unsigned char* mask)
{
    LBM_DISPATCH(c, build_links(c, mask));
}

lbm_status wall_force_any(lbm_ctx* c)
{
    LBM_DISPATCH(c, wall_force(c));
}

}  // namespace

extern "C" {

lbm_status lbm_create(lbm_ctx** out, lbm_lattice lattice, int nx, int ny, int nz, double tau,
                      const double force[3], const lbm_bc* bc, lbm_storage storage, unsigned flags)
{
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (lattice != LBM_D2Q9 && lattice != LBM_D3Q19 && lattice != LBM_D3Q27)
        return fail(LBM_EINVAL, "unknown lattice %d", int(lattice));
    if (storage_size(storage) == 0) return fail(LBM_EINVAL, "unknown storage %d", int(storage));
    if (flags & ~unsigned(LBM_FLAG_AA | LBM_FLAG_GRAPH)) return fail(LBM_EINVAL, "unknown flags 0x%x", flags);
    const int n[3] = {nx, ny, nz};
    int b[3] = {LBM_PERIODIC, LBM_PERIODIC, LBM_PERIODIC};
    if (bc)
        for (int d = 0; d < 3; ++d) b[d] = bc->axis[d];
    double F[3] = {0.0, 0.0, 0.0};
    if (force)
        for (int d = 0; d < 3; ++d) F[d] = force[d];
    for (int d = 0; d < 3; ++d) {
        if (n[d] < 1 || n[d] > 65535) return fail(LBM_EINVAL, "dimension %d = %d outside [1, 65535]", d, n[d]);
        if (b[d] != LBM_PERIODIC && b[d] != LBM_SOLID_ENDS && b[d] != LBM_WALLS_OUTSIDE)
            return fail(LBM_EINVAL, "unknown boundary %d on axis %d", b[d], d);
        if (b[d] == LBM_SOLID_ENDS && n[d] < 3)
            return fail(LBM_EINVAL, "axis %d has solid ends and needs >= 3 nodes", d);
        if (!std::isfinite(F[d])) return fail(LBM_EINVAL, "force component %d is not finite", d);
    }
    if (lattice == LBM_D2Q9 && (nz != 1 || b[2] != LBM_PERIODIC || F[2] != 0.0))
        return fail(LBM_EINVAL, "D2Q9 needs nz = 1, periodic z and F_z = 0");
    if (!(tau > 0.5)) return fail(LBM_EINVAL, "tau = %g must exceed 1/2", tau);
    const bool has_force = F[0] != 0.0 || F[1] != 0.0 || F[2] != 0.0;
    if (std::isinf(tau) && has_force) return fail(LBM_EINVAL, "tau = inf (pure streaming) needs F = 0");
    const unsigned long long N = (unsigned long long)nx * ny * nz;
    if (N >= (1ull << 31)) return fail(LBM_EINVAL, "nx*ny*nz = %llu must be < 2^31", N);

    lbm_ctx* c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(LBM_EINVAL, "out of host memory");
    c->lattice = lattice;
    c->D = lattice == LBM_D2Q9 ? 2 : 3;
    c->Q = lattice == LBM_D2Q9 ? 9 : (lattice == LBM_D3Q19 ? 19 : 27);
    c->nx = nx;
    c->ny = ny;
    c->nz = nz;
    c->N = unsigned(N);
    c->S = tile_shift(N);
    {
        const size_t T = size_t(1) << c->S;
        c->state_elems = (size_t(N) + T - 1) / T * T * size_t(c->Q);
    }
    c->tau = tau;
    c->omega = 1.0 / tau;
    for (int d = 0; d < 3; ++d) {
        c->F[d] = F[d];
        c->bc[d] = b[d];
    }
    c->storage = storage;
    c->flags = flags;
    c->aa = flags & LBM_FLAG_AA;
    c->use_graph = flags & LBM_FLAG_GRAPH;
    c->walls = b[0] != LBM_PERIODIC || b[1] != LBM_PERIODIC || b[2] != LBM_PERIODIC;
    c->force = has_force;
    plan_launch(c);
    *out = c;
    return LBM_OK;
}

size_t lbm_buffer_bytes(const lbm_ctx* c)
{
    if (!c) return 0;
    return round256(c->state_elems * storage_size(c->storage));
}

lbm_status lbm_bind(lbm_ctx* c, void* buf_a, void* buf_b, void* hip_stream)
{
    if (!c) return fail(LBM_EINVAL, "null context");
    if (c->bound) return fail(LBM_ESTATE, "context already bound");
    lbm_status st = check_device_ptr(buf_a, "buf_a", false);
    if (st) return st;
    if (c->aa) {
        if (buf_b) return fail(LBM_EINVAL, "buf_b must be NULL with LBM_FLAG_AA");
    } else {
        st = check_device_ptr(buf_b, "buf_b", false);
        if (st) return st;
        if (buf_a == buf_b) return fail(LBM_EINVAL, "buf_a and buf_b are the same buffer");
    }
    if ((reinterpret_cast<uintptr_t>(buf_a) | reinterpret_cast<uintptr_t>(buf_b)) & 255)
        return fail(LBM_EINVAL, "population buffers must be 256-byte aligned");
    LBM_HIP(hipMalloc(&c->d_partials, sizeof(double) * (5 * size_t(kReduceBlocks) + 4)));
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&c->h_result), 4 * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipFree(c->d_partials);
        c->d_partials = nullptr;
        return hip_fail(e, "hipHostMalloc");
    }
    c->buf[0] = buf_a;
    c->buf[1] = buf_b;
    c->cur = 0;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->bound = true;
    c->state_valid = false;
    return LBM_OK;
}

lbm_status lbm_init_equilibrium(lbm_ctx* c, const double* rho, const double* u, const double* noise)
{
    lbm_status st = need_bound(c);
    if (st) return st;
    if ((st = check_device_ptr(rho, "rho", false))) return st;
    if ((st = check_device_ptr(u, "u", false))) return st;
    if ((st = check_device_ptr(noise, "noise", true))) return st;
    c->steps = 0;
    c->cur = 0;
    c->state_valid = false;
    if ((st = import_any(c, nullptr, rho, u, noise))) return st;
    c->state_valid = true;
    return LBM_OK;
}

lbm_status lbm_set_populations(lbm_ctx* c, const double* f)
{
    lbm_status st = need_bound(c);
    if (st) return st;
    if ((st = check_device_ptr(f, "f", false))) return st;
    c->steps = 0;
    c->cur = 0;
    c->state_valid = false;
    if ((st = import_any(c, f, nullptr, nullptr, nullptr))) return st;
    c->state_valid = true;
    return LBM_OK;
}

lbm_status lbm_get_populations(lbm_ctx* c, double* f)
{
    lbm_status st = need_state(c);
    if (st) return st;
    if ((st = check_device_ptr(f, "f", false))) return st;
    LBM_DISPATCH(c, export_f(c, f));
}

lbm_status lbm_step(lbm_ctx* c, int n)
{
    lbm_status st = need_state(c);
    if (st) return st;
    if (n < 0) return fail(LBM_EINVAL, "n = %d < 0", n);
    LBM_DISPATCH(c, step(c, n));
}

lbm_status lbm_moments(lbm_ctx* c, void* rho, void* u, int out_is_f32)
{
    lbm_status st = need_state(c);
    if (st) return st;
    if ((st = check_device_ptr(rho, "rho", true))) return st;
    if ((st = check_device_ptr(u, "u", true))) return st;
    if (!rho && !u) return LBM_OK;
    LBM_DISPATCH(c, moments(c, rho, u, out_is_f32));
}

lbm_status lbm_reduce(lbm_ctx* c, double* mass, double* kinetic_energy, double* umax)
{
    lbm_status st = need_state(c);
    if (st) return st;
    if ((st = reduce_launch(c))) return st;
    LBM_HIP(hipMemcpyAsync(c->h_result, c->d_partials + 5 * size_t(kReduceBlocks), 4 * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream));
    LBM_HIP(hipStreamSynchronize(c->stream));
    if (mass) *mass = c->h_result[0];
    if (kinetic_energy) *kinetic_energy = c->h_result[1];
    if (umax) *umax = c->h_result[2];
    if (c->h_result[3] != 0.0 || !std::isfinite(c->h_result[0]) || !std::isfinite(c->h_result[1]))
        return fail(LBM_EUNSTABLE, "%.0f non-finite populations", c->h_result[3]);
    return LBM_OK;
}

long long lbm_steps_taken(const lbm_ctx* c) { return c ? c->steps : -1; }

lbm_status lbm_set_solid(lbm_ctx* c, const unsigned char* solid)
{
    lbm_status st = need_bound(c);
    if (st) return st;
    if ((st = check_device_ptr(solid, "solid", false))) return st;
    if (c->graph_exec) return fail(LBM_ESTATE, "lbm_set_solid after a graph was captured");
    if (!c->links) LBM_HIP(hipMalloc(&c->links, sizeof(unsigned) * size_t(c->N)));
    c->walls = true;
    c->state_valid = false;
    return build_links_any(c, solid);
}

lbm_status lbm_wall_force(lbm_ctx* c, double force[3])
{
    lbm_status st = need_state(c);
    if (st) return st;
    if (!force) return fail(LBM_EINVAL, "force is NULL");
    if ((st = wall_force_any(c))) return st;
    LBM_HIP(hipMemcpyAsync(c->h_result, c->d_partials + 5 * size_t(kReduceBlocks), 3 * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream));
    LBM_HIP(hipStreamSynchronize(c->stream));
    for (int d = 0; d < 3; ++d) force[d] = c->h_result[d];
    return LBM_OK;
}

lbm_status lbm_forward_record(lbm_ctx* c, int n, int k, void* ckpt)
{
    lbm_status st = need_state(c);
    if (st) return st;
    if (c->aa) return fail(LBM_EINVAL, "checkpointed runs need the two-lattice pattern (no LBM_FLAG_AA)");
    if (n < 0 || k < 1 || n % k != 0) return fail(LBM_EINVAL, "need n >= 0, k >= 1 and k dividing n (n=%d k=%d)", n, k);
    if (n == 0) return LBM_OK;
    if ((st = check_device_ptr(ckpt, "ckpt", false))) return st;
    const size_t bytes = lbm_buffer_bytes(c);
    char* ck = static_cast<char*>(ckpt);
    for (int s = 0; s < n / k; ++s) {
        LBM_HIP(hipMemcpyAsync(ck + size_t(s) * bytes, c->buf[c->cur], bytes, hipMemcpyDeviceToDevice,
                               c->stream));
        if ((st = lbm_step(c, k))) return st;
    }
    return LBM_OK;
}

size_t lbm_adjoint_workspace_bytes(const lbm_ctx* c, int k)
{
    if (!c || k < 1) return 0;
    return workspace_layout(c, k).total;
}

lbm_status lbm_adjoint(lbm_ctx* c, int n, int k, const void* ckpt, void* work, const double* u0,
                       const double* dJ_du, double* dJ_du0, double* dJ_dtau, double dJ_dforce[3])
{
    lbm_status st = need_bound(c);
    if (st) return st;
    if (c->aa) return fail(LBM_EINVAL, "the adjoint needs the two-lattice pattern (no LBM_FLAG_AA)");
    if (n < 0 || k < 1 || n % k != 0) return fail(LBM_EINVAL, "need n >= 0, k >= 1 and k dividing n (n=%d k=%d)", n, k);
    if (std::isinf(c->tau)) return fail(LBM_EINVAL, "the adjoint needs a finite tau");
    if (n > 0 && (st = check_device_ptr(ckpt, "ckpt", false))) return st;
    if ((st = check_device_ptr(work, "work", false))) return st;
    if ((st = check_device_ptr(u0, "u0", false))) return st;
    if ((st = check_device_ptr(dJ_du, "dJ_du", false))) return st;
    if ((st = check_device_ptr(dJ_du0, "dJ_du0", false))) return st;
    if (reinterpret_cast<uintptr_t>(work) & 255) return fail(LBM_EINVAL, "work must be 256-byte aligned");
    double out[4];
    if ((st = adjoint_any(c, n, k, ckpt, work, u0, dJ_du, dJ_du0, c->h_result))) return st;
    for (int i = 0; i < 4; ++i) out[i] = c->h_result[i];
    if (dJ_dtau) *dJ_dtau = out[0];
    if (dJ_dforce)
        for (int d = 0; d < 3; ++d) dJ_dforce[d] = out[1 + d];
    return LBM_OK;
}

lbm_status lbm_destroy(lbm_ctx* c)
{
    if (!c) return LBM_OK;
    lbm_status st = LBM_OK;
    if (c->d_partials) {
        hipError_t e = hipFree(c->d_partials);
        if (e != hipSuccess) st = hip_fail(e, "hipFree");
    }
    if (c->h_result) {
        hipError_t e = hipHostFree(c->h_result);
        if (e != hipSuccess) st = hip_fail(e, "hipHostFree");
    }
    if (c->links) (void)hipFree(c->links);
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    delete c;
    return st;
}

const char* lbm_status_string(lbm_status s)
{
    switch (s) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOTBOUND: return "no buffers bound";
    case LBM_EHIP: return "HIP runtime error";
    case LBM_EUNSTABLE: return "non-finite populations";
    case LBM_ESTATE: return "invalid state";
    }
    return "unknown status";
}

const char* lbm_last_error(void) { return g_last_error; }

}  // extern "C"
