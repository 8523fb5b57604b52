// Host-side context of liblbm.so shared by the per-lattice translation units:
// the lbm_ctx structure, error reporting, launch parameters and the table of
// per-(lattice, storage) operations.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "../../include/lbm.h"
#include "adjoint.hpp"
#include "kernels.hpp"

namespace imexlbm {

// Records the detail text of an error for lbm_last_error and returns st.
lbm_status fail(lbm_status st, const char* fmt, ...);
lbm_status hip_fail(hipError_t e, const char* what);

#define LBM_HIP(call)                                      \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return hip_fail(e_, #call);  \
    } while (0)

inline size_t storage_size(lbm_storage s)
{
    switch (s) {
    case LBM_F64: return 8;
    case LBM_F32: return 4;
    case LBM_F16_DEV:
    case LBM_BF16_DEV:
    case LBM_E4M11_DEV: return 2;
    }
    return 0;
}

// Steps per captured graph (even, so a replay returns the two-lattice
// buffers and the AA parity to where they started).
constexpr int kGraphSteps = 32;

// Non-temporal stores (and unshared loads) in the step kernels; the stores
// of a work-item's own nodes also carry the sc1 bit (WaveStores).
constexpr bool kNtStores = true;

struct Ops;

}  // namespace imexlbm

struct lbm_ctx {
    const imexlbm::Ops* ops = nullptr;  // kernels of this lattice and storage
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
    bool comp = false;  // compressible equilibrium (LBM_FLAG_COMPRESSIBLE)
    int nodal = -1;     // axis with LBM_WALLS_NODAL, or -1

    bool bound = false;
    int device = -1;  // current device at lbm_bind
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
    // Periodic FP64 two-lattice steps with two nodes per work-item (even nx).
    bool pairs = false;
    int pairs_shift = 7;
    dim3 pairs_grid;
    // Rows lie inside one tile and wavefronts inside one row (nx a power of
    // two, 64 <= nx <= tile length): the one-node AB step of a box without
    // walls may take k_step_ab_rows (FP32 and e4m11 storage).
    bool rows = false;
    // Rows of more than one workgroup and ny a multiple of 8: the one-node AB
    // steps run on grid_xcd, with each row's workgroups on one XCD.
    bool xcd_rows = false;
    dim3 grid_xcd;

    // Rows per segment of the streamed D2Q9 launches (0: not planned yet).
    int stream_rows = 0;

    // LBM_FLAG_GRAPH: kGraphSteps steps captured once, replayed by lbm_step.
    bool use_graph = false;
    hipStream_t capture_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
};

namespace imexlbm {

// Operations of one lattice and storage (Impl<L, S> in impl.hpp).
struct Ops {
    lbm_status (*step)(lbm_ctx*, int n);
    lbm_status (*import)(lbm_ctx*, const double* f, const double* rho, const double* u,
                         const double* noise);
    lbm_status (*export_f)(lbm_ctx*, double* f);
    lbm_status (*moments)(lbm_ctx*, void* rho, void* u, int f32);
    lbm_status (*reduce)(lbm_ctx*, double* partials);  // partials: 5 kReduceBlocks + 4 doubles
    lbm_status (*adjoint)(lbm_ctx*, int n, int k, const void* ckpt, void* ws, const double* rho0,
                          const double* u0, const double* ubar, double* u0bar, double* out4);
    lbm_status (*build_links)(lbm_ctx*, const unsigned char* mask);
    lbm_status (*wall_force)(lbm_ctx*);
    lbm_status (*step_between)(lbm_ctx*, const void* src, void* dst);
};

// Tables of each lattice kind (one translation unit each); null for an
// unknown storage.
const Ops* ops_d2q9(lbm_storage s);
const Ops* ops_d3q19(lbm_storage s);
const Ops* ops_d3q27(lbm_storage s);

inline Dims dims_of(const lbm_ctx* c)
{
    Dims g;
    g.nx = c->nx;
    g.ny = c->ny;
    g.nz = c->nz;
    for (int d = 0; d < 3; ++d) g.bc[d] = c->bc[d];
    g.N = c->N;
    g.S = c->S;
    g.links = c->links;
    g.nodal = c->nodal;
    return g;
}

// The gather mode of the current state (AA parity after an odd number of
// steps means the next step is odd).
inline int state_mode(const lbm_ctx* c)
{
    if (!c->aa) return kPull;
    return (c->steps & 1) ? kPullFlip : kLocal;
}

inline IoArgs io_args(const lbm_ctx* c)
{
    IoArgs p;
    p.g = dims_of(c);
    p.bx_shift = c->bx_shift;
    p.mode = state_mode(c);
    p.comp = c->comp ? 1 : 0;
    for (int d = 0; d < 3; ++d) p.F[d] = c->F[d];
    return p;
}

template <class C>
inline StepArgs<C> step_args(const lbm_ctx* c)
{
    StepArgs<C> p;
    p.g = dims_of(c);
    p.bx_shift = c->bx_shift;
    p.xcd_rows = 0;  // launches on grid_xcd set it
    p.c.omega = C(c->omega);
    for (int d = 0; d < 3; ++d) p.c.F[d] = C(c->F[d]);
    const double half = 1.0 - 0.5 * c->omega;
    p.c.k3 = C(3.0 * half);
    p.c.k9 = C(9.0 * half);
    return p;
}

inline size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// Byte offsets inside the lbm_adjoint workspace.
struct WorkspaceLayout {
    size_t state_bytes;  // one stored state (also the checkpoint stride)
    size_t seg, lam0, lam1, acc, result, total;
    size_t nblocks, acc_doubles;
};


inline WorkspaceLayout workspace_layout(const lbm_ctx* c, int k)
{
    WorkspaceLayout L;
    const size_t elem = storage_size(c->storage);
    const size_t celem = c->storage == LBM_F64 ? 8 : 4;  // arithmetic type of lambda
    L.state_bytes = round256(c->state_elems * elem);
    L.nblocks = size_t(c->grid.x) * c->grid.y * c->grid.z;
    L.acc_doubles = L.nblocks * kAccSlots;
    L.seg = 0;
    // k-1 recomputed states, and the final state for the compressible seed
    L.lam0 = L.seg + size_t(k - 1 + (c->comp ? 1 : 0)) * L.state_bytes;
    L.lam1 = L.lam0 + round256(c->state_elems * celem);
    L.acc = L.lam1 + round256(c->state_elems * celem);
    L.result = L.acc + round256(L.acc_doubles * sizeof(double));
    L.total = L.result + 256;
    return L;
}

}  // namespace imexlbm
