// liblbm.so: host runtime and C interface (include/lbm.h) of the gfx950 LBM
// time step.  Validates arguments, owns the context and calls the
// operations table of the context's lattice and storage (impl.hpp, one
// translation unit per lattice kind) on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "context.hpp"

using namespace imexlbm;

namespace imexlbm {

namespace {
thread_local char g_last_error[512] = "";
}  // namespace

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

}  // namespace imexlbm

namespace {

// Tile length of the stored state: 4096 nodes (the fastest of 256..8192
// measured on MI355X for D3Q19 FP64 and FP16), or N rounded up to a power of
// two for smaller boxes.
int tile_shift(unsigned long long N)
{
    int s = 0;
    while (s < 12 && (1ull << s) < N) ++s;
    return s;
}

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
    c->xcd_rows = c->grid.x > 1 && c->ny % 8 == 0;  // then bx = 256, one row per workgroup
    if (c->xcd_rows) c->grid_xcd = dim3(c->grid.x * 8, unsigned(c->ny / 8), c->nz);

    // Two nodes per work-item: nx/2 work-items per row.  Only on boxes of at
    // least 2^20 nodes (a small box is bound by launch latency and runs
    // faster with twice the workgroups of the one-node kernel) and not for
    // D3Q27, whose 54 populations per work-item cost more occupancy than the
    // wider accesses gain (measured 2-4 % slower).
    c->pairs = c->storage == LBM_F64 && c->lattice != LBM_D3Q27 && c->nx % 2 == 0 &&
               c->N >= (1u << 20);
    c->rows = c->nx >= 64 && (c->nx & (c->nx - 1)) == 0 && c->nx <= (1 << c->S);
    if (c->pairs) {
        const int half = c->nx / 2;
        int lanes = 1, s2 = 0;
        while (lanes < half && lanes < 256) {
            lanes <<= 1;
            ++s2;
        }
        const int rows = 256 / lanes;
        c->pairs_shift = s2;
        c->pairs_grid = dim3((half + lanes - 1) / lanes, (c->ny + rows - 1) / rows, c->nz);
    }
}

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

// Checks that p is device (or managed) memory on the current device and,
// when bytes > 0, that the allocation holding p extends at least bytes past
// it, so that no kernel of the call can touch memory outside it.
lbm_status check_device_ptr(const void* p, const char* name, bool allow_null, size_t bytes = 0)
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
    if (bytes > 0) {
        hipDeviceptr_t base = nullptr;
        size_t size = 0;
        e = hipMemGetAddressRange(&base, &size, const_cast<void*>(p));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(LBM_EINVAL, "%s: the allocation holding it is unknown", name);
        }
        const size_t offset = static_cast<size_t>(static_cast<const char*>(p) - static_cast<const char*>(base));
        if (offset > size || size - offset < bytes)
            return fail(LBM_EINVAL, "%s holds %zu bytes from the pointer, the call needs %zu", name,
                        offset > size ? size_t(0) : size - offset, bytes);
    }
    return LBM_OK;
}

// Device scratch of lbm_reduce_noalloc: the Monitor's per-workgroup
// partials (5 doubles for each of the kReduceBlocks workgroups, which stride
// over the whole box, so every box size fits) and the 4 results.  Each device
// holds its own copy until the process ends; calls on one device share it.
constexpr size_t kScratchDoubles = 5 * size_t(kReduceBlocks) + 4;
static __device__ __align__(256) double scratch[kScratchDoubles];

// Device address of `scratch` per device, looked up once per device by the
// first lbm_reduce_noalloc call made with that device current.  In host code
// the name `scratch` is only a host-side stand-in; kernels get this address.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_addr[kMaxDevices] = {};

lbm_status scratch_address(int dev, double** out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(LBM_EINVAL, "device %d outside [0, %d)", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_addr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(LBM_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_addr[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch_addr[dev];
    return LBM_OK;
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
    if (flags & ~unsigned(LBM_FLAG_AA | LBM_FLAG_GRAPH | LBM_FLAG_COMPRESSIBLE))
        return fail(LBM_EINVAL, "unknown flags 0x%x", flags);
    const int n[3] = {nx, ny, nz};
    int b[3] = {LBM_PERIODIC, LBM_PERIODIC, LBM_PERIODIC};
    if (bc)
        for (int d = 0; d < 3; ++d) b[d] = bc->axis[d];
    double F[3] = {0.0, 0.0, 0.0};
    if (force)
        for (int d = 0; d < 3; ++d) F[d] = force[d];
    int nodal = -1;
    for (int d = 0; d < 3; ++d) {
        if (n[d] < 1 || n[d] > 65535) return fail(LBM_EINVAL, "dimension %d = %d outside [1, 65535]", d, n[d]);
        if (b[d] != LBM_PERIODIC && b[d] != LBM_SOLID_ENDS && b[d] != LBM_WALLS_OUTSIDE &&
            b[d] != LBM_WALLS_NODAL)
            return fail(LBM_EINVAL, "unknown boundary %d on axis %d", b[d], d);
        if ((b[d] == LBM_SOLID_ENDS || b[d] == LBM_WALLS_NODAL) && n[d] < 3)
            return fail(LBM_EINVAL, "axis %d has solid ends or nodal walls and needs >= 3 nodes", d);
        if (b[d] == LBM_WALLS_NODAL) {
            if (nodal >= 0) return fail(LBM_EINVAL, "nodal walls on more than one axis");
            nodal = d;
        }
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
    c->ops = lattice == LBM_D2Q9 ? ops_d2q9(storage)
             : (lattice == LBM_D3Q19 ? ops_d3q19(storage) : ops_d3q27(storage));
    c->flags = flags;
    c->aa = flags & LBM_FLAG_AA;
    c->use_graph = flags & LBM_FLAG_GRAPH;
    c->walls = b[0] != LBM_PERIODIC || b[1] != LBM_PERIODIC || b[2] != LBM_PERIODIC;
    c->force = has_force;
    c->comp = flags & LBM_FLAG_COMPRESSIBLE;
    c->nodal = nodal;
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
    const size_t bb = lbm_buffer_bytes(c);
    lbm_status st = check_device_ptr(buf_a, "buf_a", false, bb);
    if (st) return st;
    if (c->aa) {
        if (buf_b) return fail(LBM_EINVAL, "buf_b must be NULL with LBM_FLAG_AA");
    } else {
        st = check_device_ptr(buf_b, "buf_b", false, bb);
        if (st) return st;
        if (buf_a == buf_b) return fail(LBM_EINVAL, "buf_a and buf_b are the same buffer");
    }
    if ((reinterpret_cast<uintptr_t>(buf_a) | reinterpret_cast<uintptr_t>(buf_b)) & 255)
        return fail(LBM_EINVAL, "population buffers must be 256-byte aligned");
    int dev = -1;
    LBM_HIP(hipGetDevice(&dev));
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
    c->device = dev;
    c->bound = true;
    c->state_valid = false;
    return LBM_OK;
}

lbm_status lbm_init_equilibrium(lbm_ctx* c, const double* rho, const double* u, const double* noise)
{
    lbm_status st = need_bound(c);
    if (st) return st;
    const size_t field = sizeof(double) * size_t(c->N);
    if ((st = check_device_ptr(rho, "rho", false, field))) return st;
    if ((st = check_device_ptr(u, "u", false, 3 * field))) return st;
    if ((st = check_device_ptr(noise, "noise", true, size_t(c->Q) * field))) return st;
    c->steps = 0;
    c->cur = 0;
    c->state_valid = false;
    if ((st = c->ops->import(c, nullptr, rho, u, noise))) return st;
    c->state_valid = true;
    return LBM_OK;
}

lbm_status lbm_set_populations(lbm_ctx* c, const double* f)
{
    lbm_status st = need_bound(c);
    if (st) return st;
    if ((st = check_device_ptr(f, "f", false, sizeof(double) * size_t(c->Q) * c->N))) return st;
    c->steps = 0;
    c->cur = 0;
    c->state_valid = false;
    if ((st = c->ops->import(c, f, nullptr, nullptr, nullptr))) return st;
    c->state_valid = true;
    return LBM_OK;
}

lbm_status lbm_get_populations(lbm_ctx* c, double* f)
{
    lbm_status st = need_state(c);
    if (st) return st;
    if ((st = check_device_ptr(f, "f", false, sizeof(double) * size_t(c->Q) * c->N))) return st;
    return c->ops->export_f(c, f);
}

lbm_status lbm_step(lbm_ctx* c, int n)
{
    lbm_status st = need_state(c);
    if (st) return st;
    if (n < 0) return fail(LBM_EINVAL, "n = %d < 0", n);
    return c->ops->step(c, n);
}

lbm_status lbm_moments(lbm_ctx* c, void* rho, void* u, int out_is_f32)
{
    lbm_status st = need_state(c);
    if (st) return st;
    const size_t field = (out_is_f32 ? sizeof(float) : sizeof(double)) * size_t(c->N);
    if ((st = check_device_ptr(rho, "rho", true, field))) return st;
    if ((st = check_device_ptr(u, "u", true, 3 * field))) return st;
    if (!rho && !u) return LBM_OK;
    return c->ops->moments(c, rho, u, out_is_f32);
}

lbm_status lbm_reduce(lbm_ctx* c, double* mass, double* kinetic_energy, double* umax)
{
    lbm_status st = need_state(c);
    if (st) return st;
    if ((st = c->ops->reduce(c, c->d_partials))) return st;
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

lbm_status lbm_reduce_noalloc(lbm_ctx* c, double* result)
{
    lbm_status st = need_state(c);
    if (st) return st;
    static_assert(kScratchDoubles >= 5 * size_t(kReduceBlocks) + 4, "scratch too small for the partials");
    const size_t need = 5 * size_t(kReduceBlocks) + 4;  // the same for every box size
    if (need > kScratchDoubles)
        return fail(LBM_EINVAL, "the reduction needs %zu doubles of scratch, the maximum is %zu", need,
                    kScratchDoubles);
    if ((st = check_device_ptr(result, "result", false, 4 * sizeof(double)))) return st;
    int dev = -1;
    LBM_HIP(hipGetDevice(&dev));
    if (dev != c->device)
        return fail(LBM_EINVAL, "current device %d is not the device %d the context was bound on", dev,
                    c->device);
    double* ptr = nullptr;
    if ((st = scratch_address(dev, &ptr))) return st;
    if ((st = c->ops->reduce(c, ptr))) return st;
    LBM_HIP(hipMemcpyAsync(result, ptr + 5 * size_t(kReduceBlocks), 4 * sizeof(double), hipMemcpyDeviceToDevice,
                           c->stream));
    return LBM_OK;
}

long long lbm_steps_taken(const lbm_ctx* c) { return c ? c->steps : -1; }

lbm_status lbm_set_solid(lbm_ctx* c, const unsigned char* solid)
{
    lbm_status st = need_bound(c);
    if (st) return st;
    if ((st = check_device_ptr(solid, "solid", false, size_t(c->N)))) return st;
    if (c->graph_exec) return fail(LBM_ESTATE, "lbm_set_solid after a graph was captured");
    if (!c->links) LBM_HIP(hipMalloc(&c->links, sizeof(unsigned) * size_t(c->N)));
    c->walls = true;
    c->state_valid = false;
    return c->ops->build_links(c, solid);
}

lbm_status lbm_wall_force(lbm_ctx* c, double force[3])
{
    lbm_status st = need_state(c);
    if (st) return st;
    if (!force) return fail(LBM_EINVAL, "force is NULL");
    if ((st = c->ops->wall_force(c))) return st;
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
    const size_t bytes = lbm_buffer_bytes(c);
    if ((st = check_device_ptr(ckpt, "ckpt", false, size_t(n / k) * bytes))) return st;
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

lbm_status lbm_adjoint(lbm_ctx* c, int n, int k, const void* ckpt, void* work, const double* rho0,
                       const double* u0, const double* dJ_du, double* dJ_du0, double* dJ_dtau,
                       double dJ_dforce[3])
{
    lbm_status st = need_bound(c);
    if (st) return st;
    if (c->aa) return fail(LBM_EINVAL, "the adjoint needs the two-lattice pattern (no LBM_FLAG_AA)");
    if (n < 0 || k < 1 || n % k != 0) return fail(LBM_EINVAL, "need n >= 0, k >= 1 and k dividing n (n=%d k=%d)", n, k);
    if (std::isinf(c->tau)) return fail(LBM_EINVAL, "the adjoint needs a finite tau");
    if (c->comp && n < 1) return fail(LBM_EINVAL, "the compressible adjoint needs n >= 1");
    const size_t field = sizeof(double) * size_t(c->N);
    if (c->comp && (st = check_device_ptr(rho0, "rho0", false, field))) return st;
    if (n > 0 && (st = check_device_ptr(ckpt, "ckpt", false, size_t(n / k) * lbm_buffer_bytes(c)))) return st;
    if ((st = check_device_ptr(work, "work", false, lbm_adjoint_workspace_bytes(c, k)))) return st;
    if ((st = check_device_ptr(u0, "u0", false, 3 * field))) return st;
    if ((st = check_device_ptr(dJ_du, "dJ_du", false, 3 * field))) return st;
    if ((st = check_device_ptr(dJ_du0, "dJ_du0", false, 3 * field))) return st;
    if (reinterpret_cast<uintptr_t>(work) & 255) return fail(LBM_EINVAL, "work must be 256-byte aligned");
    double out[4];
    if ((st = c->ops->adjoint(c, n, k, ckpt, work, rho0, u0, dJ_du, dJ_du0, c->h_result))) return st;
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
