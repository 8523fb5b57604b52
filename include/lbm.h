/*
 * lbm.h -- C interface of liblbm.so, the gfx950 (MI355X) implementation of
 * the lattice Boltzmann time step of IMEXLBM (Liu, Patel, Balakrishnan, Lee,
 * "IMEXLBM 1.0: A Proxy Application based on the Lattice Boltzmann Method
 * for solving CFD problems on GPUs", 2022).
 *
 * The calls follow the paper's program structure (Sec. 3.1):
 *   lbm_create           DataInput + InitLattice + SetGeometry (Sec. 3.1, Table 4)
 *   lbm_bind             AllocateArrays / TARGET ENTER DATA: the caller's device
 *                        buffers and stream become the state of the context
 *   lbm_init_equilibrium InitUP + InitPDF: f = feq(rho, u) (Sec. 2.2)
 *   lbm_step             n passes of Collision -> BoundaryCondition ->
 *                        Propagation -> PostProcessing (Sec. 3.1; Eqs.
 *                        (collision), (bb), (propagation))
 *   lbm_moments          PostProcessing outputs p/c_s^2 and u (Sec. 2.1)
 *   lbm_reduce           Monitor (Sec. 3.6): global reductions
 *   lbm_destroy          DeAllocateArrays / TARGET EXIT DATA
 *
 * Conventions shared by every call:
 *   - A "field" is a device array in the canonical structure-of-arrays order
 *     [component][z][y][x], x fastest, N = nx*ny*nz nodes per component:
 *     rho is [N], u is [3][N] (u_z = 0 for D2Q9), populations are [Q][N].
 *   - tau is the lattice relaxation time: omega = 1/tau, nu = (tau - 1/2)/3.
 *     The paper's tau (Eq. (collision), relaxation parameter
 *     1/(tau/dt + 1/2), dt = 1) is this tau minus 1/2.
 *   - "rho" is p/c_s^2 = sum_a f_a, the quantity the Collision listing uses
 *     as 3p (Sec. 3.6); c_s^2 = 1/3 and rho0 = 1 (Table 3).
 *   - The velocity is u = (sum_a e_a f_a + F/2)/rho0: the incompressible
 *     model's moment (Sec. 2.1) shifted by half the body force F, which
 *     enters the collision as t_a [3 (e_a - u).F + 9 (e_a.u)(e_a.F)] times
 *     (1 - omega/2) (trapezoidal forcing; the paper gives no force term).
 *     The equilibrium is the incompressible one of Eq. (incompressible_feq),
 *     t_a [rho + rho0 (3 e.u + 4.5 (e.u)^2 - 1.5 u.u)], unless
 *     LBM_FLAG_COMPRESSIBLE selects the weakly compressible one of Eq.
 *     (feq), t_a rho [1 + 3 e.u + 4.5 (e.u)^2 - 1.5 u.u], with
 *     u = (sum_a e_a f_a + F/2)/rho.
 *   - Walls are halfway bounce-back (Eq. (bb)): a population whose pull
 *     source x - e_a is solid is replaced by the opposite population of the
 *     same node.  Solid nodes carry no state.  LBM_WALLS_NODAL gives the
 *     modified nodal variant of Sec. 2.2 instead.
 *   - The caller owns every device buffer and the stream (e.g. torch tensors
 *     and torch's current stream); they must outlive their use by the
 *     context.  The library owns the context and a small device scratch for
 *     reductions, allocated in lbm_bind and freed in lbm_destroy.
 *   - Every call returns LBM_OK (0) or a negative lbm_status and never
 *     throws.  Arguments are checked on the host before any launch; a
 *     device pointer must be device (or managed) memory of the current
 *     device whose allocation extends at least as far past the pointer as
 *     the call reads or writes (LBM_EINVAL otherwise).  A HIP
 *     failure returns LBM_EHIP; lbm_last_error() then holds the HIP error
 *     text.  Kernel faults are asynchronous and surface at the next call
 *     that synchronises.  A context is not thread-safe; separate contexts
 *     are independent.
 */
#ifndef IMEXLBM_LBM_H
#define IMEXLBM_LBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,    /* bad argument; nothing was launched */
    LBM_ENOTBOUND = -2, /* call needs lbm_bind first */
    LBM_EHIP = -3,      /* HIP runtime error (text in lbm_last_error) */
    LBM_EUNSTABLE = -4, /* lbm_reduce found a non-finite population */
    LBM_ESTATE = -5     /* call not valid in the context's current state */
} lbm_status;

/* Discrete velocity models of Sec. 2.1.  D2Q9 is numbered as printed there
 * (lexicographic in (e_x, e_y), e_x slowest); D3Q27 extends that rule to
 * all of {-1,0,1}^3 (the lattice of the paper's validation case, Sec. 5) and
 * D3Q19 is that order without the 8 corners.  In each the opposite of a is
 * Q - 1 - a. */
typedef enum { LBM_D2Q9 = 0, LBM_D3Q19 = 1, LBM_D3Q27 = 2 } lbm_lattice;

/* Storage of the populations in device memory.  LBM_F64 stores f and
 * computes in FP64 (the paper's precision).  The others store the deviation
 * f_a - t_a and compute in FP32: LBM_F32 in FP32, LBM_F16_DEV in IEEE half,
 * LBM_BF16_DEV in bfloat16, LBM_E4M11_DEV in a 16-bit format with 4 exponent
 * and 11 fraction bits (after the FP16C format of Lehmann et al., Phys. Rev.
 * E 106, 015308 (2022): |f_a - t_a| < 1, so the exponent range of IEEE half
 * is traded for one more fraction bit; normal numbers 2^-14 .. 0.99976,
 * subnormals down to 2^-25, IEEE-style infinities and NaN; twice the
 * precision of IEEE half everywhere below 1), each rounded to nearest-even
 * on store.  Reductions accumulate in FP64 for every storage. */
typedef enum {
    LBM_F64 = 0,
    LBM_F32 = 1,
    LBM_F16_DEV = 2,
    LBM_BF16_DEV = 3,
    LBM_E4M11_DEV = 4
} lbm_storage;

/* Boundary of one axis. */
typedef enum {
    LBM_PERIODIC = 0,      /* wrap-around, done inside the kernels */
    LBM_SOLID_ENDS = 1,    /* first and last planes are solid nodes; walls
                              lie half a cell inside them */
    LBM_WALLS_OUTSIDE = 2, /* every plane is fluid; walls lie half a cell
                              outside the first and last planes */
    LBM_WALLS_NODAL = 3    /* modified nodal bounce-back (Sec. 2.2): the first
                              and last planes are wall nodes that collide like
                              the bulk; after each propagation a population of
                              a wall node whose source lies beyond the wall is
                              a copy of the opposite one (Eq. (bb)).  One axis
                              at most; wall force excludes these walls */
} lbm_axis_bc;

typedef struct {
    int axis[3]; /* lbm_axis_bc for x, y, z */
} lbm_bc;

/* lbm_create flags. */
enum {
    LBM_FLAG_AA = 1,           /* in-place AA pattern: one population buffer instead of two */
    LBM_FLAG_GRAPH = 2,        /* lbm_step replays a HIP graph of 32 captured steps (captured
                                  on first use on a private stream, launched on the bound
                                  stream): fewer launch round trips for small, launch-bound
                                  boxes */
    LBM_FLAG_COMPRESSIBLE = 4  /* weakly compressible equilibrium of Eq. (feq), u = j/rho */
};

/*
 * Creates a context for an nx*ny*nz box.  Checks (LBM_EINVAL otherwise):
 * tau > 1/2 (tau = +inf is pure streaming, allowed only with F = 0);
 * every dimension >= 1 and >= 3 on an LBM_SOLID_ENDS or LBM_WALLS_NODAL
 * axis; LBM_WALLS_NODAL on one axis at most; D2Q9 needs nz = 1, a periodic
 * z axis and F_z = 0; F finite; N = nx*ny*nz < 2^31; flags only
 * LBM_FLAG_AA, LBM_FLAG_GRAPH and LBM_FLAG_COMPRESSIBLE.  force may be NULL
 * (no force); bc may be NULL (fully periodic).  No device work happens
 * here.
 */
lbm_status lbm_create(lbm_ctx** out, lbm_lattice lattice, int nx, int ny, int nz, double tau,
                      const double force[3], const lbm_bc* bc, lbm_storage storage,
                      unsigned flags);

/* Bytes of one population buffer: the nodes in tiles of T = 4096 (fewer,
 * a power of two, for boxes under 4096 nodes), Q runs of T storage elements
 * per tile, whole tiles; a multiple of 256. */
size_t lbm_buffer_bytes(const lbm_ctx* ctx);

/*
 * Binds device memory and a stream.  buf_a and buf_b are two population
 * buffers of lbm_buffer_bytes() each (buf_b must be NULL with LBM_FLAG_AA
 * and non-NULL otherwise), 256-byte aligned, on the current device.
 * hip_stream is a hipStream_t (NULL = the null stream); every later launch
 * goes to it, in order.  Allocates the reduction scratch.  The state is
 * undefined until lbm_init_equilibrium or lbm_set_populations.
 */
lbm_status lbm_bind(lbm_ctx* ctx, void* buf_a, void* buf_b, void* hip_stream);

/*
 * InitPDF: f_a = t_a [rho + rho0 (3 e_a.u + 4.5 (e_a.u)^2 - 1.5 u.u)]
 * (Eq. (incompressible_feq); with LBM_FLAG_COMPRESSIBLE the rho0 factor is
 * rho, Eq. (feq)) on every fluid node, plus noise_a if noise is not NULL.
 * On nodal wall nodes Eq. (bb) then replaces the unknown populations.
 * rho [N], u [3][N], noise [Q][N]: device FP64 fields.  Asynchronous on the
 * bound stream.
 */
lbm_status lbm_init_equilibrium(lbm_ctx* ctx, const double* rho, const double* u,
                                const double* noise);

/*
 * Sets / reads the populations f^n of the paper's f array after the last
 * Propagation (device FP64 field [Q][N]; solid nodes are ignored on set and
 * read back as 0).  For the FP64 storage the round trip is bit-exact; the
 * other storages round f - t_a on set.  On nodal wall nodes the unknown
 * populations are determined by Eq. (bb): the values set for them are
 * ignored and read back as the opposite populations.  Asynchronous on the
 * bound stream.
 */
lbm_status lbm_set_populations(lbm_ctx* ctx, const double* f);
lbm_status lbm_get_populations(lbm_ctx* ctx, double* f);

/*
 * Advances n >= 0 time steps.  Asynchronous on the bound stream.  A
 * periodic D2Q9 two-lattice box runs eight steps at a time as two launches
 * of four steps each (blocked in LDS) and the rest one launch per step;
 * the state after any n is bit for bit that of n one-step launches.
 */
lbm_status lbm_step(lbm_ctx* ctx, int n);

/*
 * PostProcessing of the current f^n: rho = sum_a f_a [N] and
 * u = (sum_a e_a f_a + F/2)/rho0 [3][N] (divided by rho instead with
 * LBM_FLAG_COMPRESSIBLE), written as FP64 (out_is_f32 = 0) or
 * FP32 (out_is_f32 = 1) device fields; either pointer may be NULL.  Solid
 * nodes read 0.  Asynchronous on the bound stream.
 */
lbm_status lbm_moments(lbm_ctx* ctx, void* rho, void* u, int out_is_f32);

/*
 * Monitor: total mass sum rho, kinetic energy (rho0/2) sum |u|^2 (sum
 * (rho/2) |u|^2 with LBM_FLAG_COMPRESSIBLE) and max |u| over the fluid
 * nodes, accumulated in FP64 in a fixed order (the
 * result does not depend on scheduling).  Host outputs, any may be NULL.
 * Synchronises the bound stream.  Returns LBM_EUNSTABLE (outputs still
 * written) when a population is NaN or infinite.
 */
lbm_status lbm_reduce(lbm_ctx* ctx, double* mass, double* kinetic_energy, double* umax);

/*
 * lbm_reduce for callers that cannot allocate memory or wait on the stream
 * (code under HIP graph capture, tight serving loops): the same Monitor
 * reduction, with the same kernels and summation order, so the results are
 * bit for bit those of lbm_reduce.  It calls no allocating routine and does
 * not synchronise: the per-workgroup partials go to a library-owned static
 * device array of 5 * 1024 + 4 doubles (41 KiB) per device, held until the
 * process ends, which is enough for every box lbm_create accepts (the
 * reduction runs a fixed grid of 1024 workgroups over the box).  result:
 * device FP64 [4] written asynchronously on the bound stream with mass,
 * kinetic energy, max |u| and the number of non-finite populations (the
 * caller checks the last one; there is no LBM_EUNSTABLE here).  The current
 * device must be the one the context was bound on (LBM_EINVAL otherwise).
 * Every call on a device shares that device's array, which keeps the last
 * call's partials: calls whose reductions overlap on one device (different
 * streams, or threads) race and may return mixed results; calls ordered on
 * one stream do not.
 */
lbm_status lbm_reduce_noalloc(lbm_ctx* ctx, double* result);

/*
 * SetGeometry with a solid mask (Sec. 3.3: the geo array marks fluid and
 * solid nodes): solid[id] != 0 makes node id solid, in addition to the solid
 * end planes of LBM_SOLID_ENDS axes.  Every link from a fluid node into a
 * solid node bounces back halfway (Eq. (bb)).  solid: device uint8 [N].
 * Call after lbm_bind and before initialising the populations (the state
 * becomes undefined); not after a graph was captured (LBM_ESTATE).  The
 * library allocates 4 bytes per node for per-node link bits (freed by
 * lbm_destroy) and the step kernels read them: 4 more bytes per update.
 * Asynchronous on the bound stream.
 */
lbm_status lbm_set_solid(lbm_ctx* ctx, const unsigned char* solid);

/*
 * Momentum-exchange force on all halfway walls (solid nodes and the box
 * walls; not LBM_WALLS_NODAL walls) during the last propagation, the drag
 * evaluation of Sec. 4:
 * F = sum over fluid x and directions a with x + e_a a wall of
 * [f*_a(x, t) + f_abar(x, t + 1)] e_a = 2 f_abar(x, t + 1) e_a (the
 * population that came back is the one that left).  Host output [3],
 * accumulated in FP64 in a fixed order.  Synchronises the bound stream.
 */
lbm_status lbm_wall_force(lbm_ctx* ctx, double force[3]);

/* Time steps taken since the last init/set (the AA parity is its low bit). */
long long lbm_steps_taken(const lbm_ctx* ctx);

/*
 * Discrete adjoint (not in the paper; the reverse-mode derivative of n time
 * steps).  Forward model: f^0 = feq(rho, u0) (+ noise) by
 * lbm_init_equilibrium, f^{k+1} = S C(f^k; tau, F) by lbm_step, and the
 * final velocity u^n = sum_a e_a f^n_a + F/2.  For a scalar J(u^n) the
 * adjoint returns dJ/du0, dJ/dtau and dJ/dF given dJ/du^n.
 *
 * In the compressible model u^n = (sum_a e_a f^n_a + F/2)/rho^n and the
 * init map's equilibrium carries the factor rho.  With LBM_WALLS_NODAL the
 * forward step includes the copy of Eq. (bb) on wall nodes.
 *
 * lbm_forward_record advances n steps from the current state like
 * lbm_step(ctx, n) and stores the state at steps 0, k, 2k, ..., n-k
 * (relative to the start) in ckpt: n/k consecutive device buffers of
 * lbm_buffer_bytes() each.  k must divide n.  Two-lattice pattern only
 * (LBM_EINVAL with LBM_FLAG_AA).  Asynchronous on the bound stream.
 */
lbm_status lbm_forward_record(lbm_ctx* ctx, int n, int k, void* ckpt);

/* Device workspace lbm_adjoint needs for checkpoint interval k: k-1 state
 * buffers for the recomputed segment (k with LBM_FLAG_COMPRESSIBLE, whose
 * output map needs the final state), two adjoint fields and the FP64
 * accumulators.  0 for a NULL context or k < 1. */
size_t lbm_adjoint_workspace_bytes(const lbm_ctx* ctx, int k);

/*
 * Backward sweep over the n steps recorded by lbm_forward_record with the
 * same n and k (ckpt as filled there, unchanged).  Each k-step segment is
 * recomputed from its checkpoint into the workspace, then k adjoint steps
 * run backwards: the transposed propagation (a pull from x + e_a, with the
 * bounce-back links reversed) and the transposed collision Jacobian.  The
 * segment recompute and the adjoint steps read the stored states; the
 * context's own buffers and state are not touched.
 *   rho0   [N] device FP64: the density given to lbm_init_equilibrium;
 *          read with LBM_FLAG_COMPRESSIBLE only (may be NULL otherwise)
 *   u0     [3][N] device FP64: the initial velocity given to
 *          lbm_init_equilibrium (the init map's linearisation point)
 *   dJ_du  [3][N] device FP64: dJ/du^n (solid nodes ignored)
 *   dJ_du0 [3][N] device FP64 output (0 on solid nodes)
 *   dJ_dtau, dJ_dforce: host outputs (either may be NULL), accumulated in
 *          FP64 in a fixed order; dJ_dforce[2] = 0 for D2Q9
 * work: lbm_adjoint_workspace_bytes(ctx, k) bytes of device memory,
 * 256-byte aligned.  Adjoint fields use the storage's arithmetic type
 * (FP64 for LBM_F64, FP32 otherwise).  Needs a finite tau and the
 * two-lattice pattern, and n >= 1 with LBM_FLAG_COMPRESSIBLE.
 * Synchronises the bound stream.
 */
lbm_status lbm_adjoint(lbm_ctx* ctx, int n, int k, const void* ckpt, void* work,
                       const double* rho0, const double* u0, const double* dJ_du, double* dJ_du0,
                       double* dJ_dtau, double dJ_dforce[3]);

/* Frees the context and its scratch (not the caller's buffers).  NULL is a
 * no-op. */
lbm_status lbm_destroy(lbm_ctx* ctx);

/* Static text for a status code. */
const char* lbm_status_string(lbm_status status);
/* Detail of the last error raised on this thread (never NULL). */
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
