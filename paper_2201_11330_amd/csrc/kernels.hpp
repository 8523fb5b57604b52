// Device code of the LBM time step for gfx950.
//
// Layout: nodes are numbered x + nx*(y + ny*z) (x fastest).  A population
// buffer is an array of tiles of T = 2^S consecutive nodes; a tile holds Q
// runs of T elements, one per direction (structure of arrays inside the
// tile, see slot()).  One work-item owns one node (two in the *_pairs
// kernels); 256-item workgroups cover a (BX x BY) tile of an x-y plane with
// BX a power of two (the full row when nx <= 256), so the 64 lanes of a
// wavefront touch 64 consecutive nodes of a row and every access is a
// coalesced 64-element run.  The 19
// loads and 19 stores of a wavefront land in a few contiguous regions
// instead of 19 separate planes (measured 4-10 % faster than plain
// structure of arrays on MI355X).
//
// Two-lattice scheme (AB): the stored state is the post-collision
// population f* of the previous step.  One launch pulls
// f_a(x) = f*_a(x - e_a) (Eq. (propagation)), or f*_abar(x) when x - e_a is
// a wall (Eq. (bb)), takes the moments, collides (Eq. (collision)) and
// writes f*(x) to the other buffer: 2*Q*sizeof(storage) bytes per node.
//
// AA pattern (one buffer): even steps read and write the node's own slots,
// writing f*_a to slot abar; odd steps read the neighbours' opposite slots
// and write back to where the next even step finds them.  A work-item
// reads and writes the same set of addresses, so the update is in place.
//
// Walls of the modified nodal scheme (Sec. 2.2) are addressed like walls
// half a cell outside the box; after the loads, the populations of a wall
// node whose source lies beyond the wall are replaced by the opposite ones
// (Eq. (bb)) before the collision, so the slots they were read from carry
// nothing (nodal_fill).
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "e4m11.hpp"
#include "lattice.hpp"

namespace imexlbm {

enum AxisBC : int { kPeriodic = 0, kSolidEnds = 1, kWallsOutside = 2, kWallsNodal = 3 };

// How a stored state maps to the paper's post-propagation f^n.
enum GatherMode : int {
    kPull = 0,      // AB state, and AA before an odd step with slots flipped
    kPullFlip = 1,  // AA before an odd step: f^n_a(x) = A[abar](x - e_a)
    kLocal = 2      // AA before an even step: f^n_a(x) = A[a](x)
};

// ---------------------------------------------------------------------------
// Storage traits: element type in memory, arithmetic type, conversions.

template <class S>
struct Store;

template <>
struct Store<double> {
    using C = double;
    static constexpr bool kDeviation = false;
    __device__ static C load(double v) { return v; }
    __device__ static double save(C v) { return v; }
};

template <>
struct Store<float> {
    using C = float;
    static constexpr bool kDeviation = true;
    __device__ static C load(float v) { return v; }
    __device__ static float save(C v) { return v; }
};

template <>
struct Store<__half> {
    using C = float;
    static constexpr bool kDeviation = true;
    __device__ static C load(__half v) { return __half2float(v); }
    __device__ static __half save(C v) { return __float2half_rn(v); }
};

template <>
struct Store<__hip_bfloat16> {
    using C = float;
    static constexpr bool kDeviation = true;
    __device__ static C load(__hip_bfloat16 v) { return __bfloat162float(v); }
    __device__ static __hip_bfloat16 save(C v) { return __float2bfloat16(v); }  // nearest-even
};

template <>
struct Store<e4m11> {
    using C = float;
    static constexpr bool kDeviation = true;
    __device__ static C load(e4m11 v) { return e4m11_to_float(v); }
    __device__ static e4m11 save(C v) { return e4m11_from_float(v); }  // nearest-even
};

// ---------------------------------------------------------------------------
// Compile-time helpers.

template <class F, int... Is>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Is...>)
{
    (f(std::integral_constant<int, Is>{}), ...);
}

// Calls f(std::integral_constant<int, a>) for a = 0..N-1.
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// e * v for a lattice component e in {-1, 0, 1}; the zero term is -0.0, the
// additive identity the compiler may drop.
template <int E, class T>
__device__ __forceinline__ T eterm(T v)
{
    if constexpr (E == 1) return v;
    else if constexpr (E == -1) return -v;
    else return T(-0.0);
}

// ---------------------------------------------------------------------------
// Geometry.

struct Dims {
    int nx, ny, nz;
    int bc[3];
    unsigned N;  // nx*ny*nz
    int S;       // log2 of the tile length T of the stored state
    // Per-node link bits when a solid mask is set (else null): bit a is set
    // when the pull source x - e_a is a wall (solid node or outside the
    // box), bit 31 when the node itself is solid.
    const unsigned* links;
    int nodal;  // axis with walls of the modified nodal scheme, or -1
};

__device__ __forceinline__ unsigned node_index(const Dims& g, int x, int y, int z)
{
    return unsigned(x) + unsigned(g.nx) * (unsigned(y) + unsigned(g.ny) * unsigned(z));
}

// Element offset of direction a of node idx in a stored state.
template <int Q>
__device__ __forceinline__ size_t slot(int a, unsigned idx, int S)
{
    return ((size_t(idx >> S) * Q + size_t(a)) << S) | (idx & ((1u << S) - 1u));
}

// Coordinates c-1, c, c+1 of one axis (index = shift + 1), wrapped on a
// periodic axis, and whether each is a wall (a solid plane, or outside the
// box).  A wall entry keeps coordinate c so its index stays in range.
struct Axis3 {
    int c[3];
    bool wall[3];
};

// A nodal-wall axis is addressed like walls outside the box.
template <bool WALLS>
__device__ __forceinline__ Axis3 axis3(int c, int n, int bc)
{
    Axis3 r;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        int s = c + k - 1;
        bool wall = false;
        if (!WALLS || bc == kPeriodic) {
            s = s < 0 ? s + n : (s >= n ? s - n : s);
        } else if (bc == kSolidEnds) {
            wall = s <= 0 || s >= n - 1;
            if (wall) s = c;
        } else {
            wall = s < 0 || s >= n;
            if (wall) s = c;
        }
        r.c[k] = s;
        r.wall[k] = wall;
    }
    return r;
}

__device__ __forceinline__ bool axis_solid(const Dims& g, int x, int y, int z)
{
    return (g.bc[0] == kSolidEnds && (x == 0 || x == g.nx - 1)) ||
           (g.bc[1] == kSolidEnds && (y == 0 || y == g.ny - 1)) ||
           (g.bc[2] == kSolidEnds && (z == 0 || z == g.nz - 1));
}

__device__ __forceinline__ bool is_solid(const Dims& g, int x, int y, int z)
{
    if (g.links) return (g.links[node_index(g, x, y, z)] >> 31) != 0u;
    return axis_solid(g, x, y, z);
}

// Node of this work-item for the (BX = 1 << bx_shift) x (256 / BX) tiling.
__device__ __forceinline__ bool node_of_item(const Dims& g, int bx_shift, int& x, int& y, int& z)
{
    const int tx = threadIdx.x & ((1 << bx_shift) - 1);
    const int ty = threadIdx.x >> bx_shift;
    x = (blockIdx.x << bx_shift) + tx;
    y = blockIdx.y * (blockDim.x >> bx_shift) + ty;
    z = blockIdx.z;
    return x < g.nx && y < g.ny;
}

// As node_of_item, for rows of more than one workgroup (BX = 256 nodes per
// workgroup, one row per workgroup), launched on the grid
// (8 G, ny / 8, nz) with G workgroups per row.  The dispatcher hands
// workgroup k (in x-fastest order) to XCD k mod 8, and k mod 8 = blockIdx.x
// mod 8 here; blockIdx.x = 8 xb + j is part xb of row 8 blockIdx.y + j, so
// the G workgroups of a row have consecutive ids among those of one XCD.
// The lines at the seams between them, which the x-shifted loads of both
// sides read, then come into one L2 instead of two.
__device__ __forceinline__ bool node_of_item_rows_on_xcd(const Dims& g, int bx_shift, int& x, int& y, int& z)
{
    const int tx = threadIdx.x & ((1 << bx_shift) - 1);
    x = int((blockIdx.x >> 3) << bx_shift) + tx;
    y = int(blockIdx.y * 8 + (blockIdx.x & 7));
    z = blockIdx.z;
    return x < g.nx;
}

// In-plane index of x + sgn*e_a for every a, and whether that node is a wall.
template <int L, bool WALLS, int SGN>
__device__ __forceinline__ void link_nodes(const Dims& g, int x, int y, int z,
                                           unsigned (&idx)[Lattice<L>::Q],
                                           bool (&wall)[Lattice<L>::Q])
{
    const Axis3 ax = axis3<WALLS>(x, g.nx, g.bc[0]);
    const Axis3 ay = axis3<WALLS>(y, g.ny, g.bc[1]);
    Axis3 az;
    if constexpr (kDim<L> == 3) {
        az = axis3<WALLS>(z, g.nz, g.bc[2]);
    } else {
        az = Axis3{{z, z, z}, {false, false, false}};
    }
    static_for<Lattice<L>::Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        constexpr int kx = 1 + SGN * kLattice<L>.e[a][0];
        constexpr int ky = 1 + SGN * kLattice<L>.e[a][1];
        constexpr int kz = 1 + SGN * kLattice<L>.e[a][2];
        idx[a] = unsigned(ax.c[kx]) + unsigned(g.nx) * (unsigned(ay.c[ky]) + unsigned(g.ny) * unsigned(az.c[kz]));
        wall[a] = WALLS && (ax.wall[kx] || ay.wall[ky] || az.wall[kz]);
    });
    if (WALLS && g.links) {
        // x + e_a is the pull source of the opposite direction.
        const unsigned bits = g.links[node_index(g, x, y, z)];
        static_for<Lattice<L>::Q>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            constexpr int bit = SGN < 0 ? a : Lattice<L>::opp(a);
            wall[a] = (bits >> bit) & 1u;
        });
    }
}

// Element offset of the slot holding f^n_a(x) in a stored state (GatherMode),
// given the pull sources of the node.  The same offsets, written instead of
// read, import a state: the map is a bijection between (node, direction)
// pairs of fluid nodes and slots.
template <int L>
__device__ __forceinline__ size_t gather_offset(int mode, int a, unsigned own, unsigned src,
                                                bool wall, int S)
{
    constexpr int Q = Lattice<L>::Q;
    const int abar = Lattice<L>::opp(a);
    if (mode == kLocal) return slot<Q>(a, own, S);
    if (mode == kPull) return wall ? slot<Q>(abar, own, S) : slot<Q>(a, src, S);
    return wall ? slot<Q>(a, own, S) : slot<Q>(abar, src, S);  // kPullFlip
}

// Eq. (bb) on a wall node of the nodal scheme: each population whose pull
// source lies beyond the wall (e along the nodal axis pointing away from
// the wall's outside) becomes a copy of the opposite population, which
// arrived from inside the box.  No-op off the wall planes.
template <int L, class C>
__device__ __forceinline__ void nodal_fill(const Dims& g, int x, int y, int z,
                                           C (&f)[Lattice<L>::Q])
{
    const int ax = g.nodal;
    if (ax < 0) return;
    const int c = ax == 0 ? x : (ax == 1 ? y : z);
    const int n = ax == 0 ? g.nx : (ax == 1 ? g.ny : g.nz);
    const int side = c == 0 ? 1 : (c == n - 1 ? -1 : 0);  // e of the unknowns
    if (side == 0) return;
    static_for<Lattice<L>::Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        constexpr auto& LT = kLattice<L>;
        const int e = ax == 0 ? LT.e[a][0] : (ax == 1 ? LT.e[a][1] : LT.e[a][2]);
        if (e == side) f[a] = f[Lattice<L>::opp(a)];
    });
}

// Whether x + sgn e_a lies beyond a wall of the nodal scheme.
template <int L, int SGN>
__device__ __forceinline__ bool beyond_nodal(const Dims& g, int x, int y, int z, int a)
{
    const int ax = g.nodal;
    if (ax < 0) return false;
    const int c = ax == 0 ? x : (ax == 1 ? y : z);
    const int n = ax == 0 ? g.nx : (ax == 1 ? g.ny : g.nz);
    const int t = c + SGN * kLattice<L>.e[a][ax];
    return t < 0 || t >= n;
}

// Loads and stores of population elements.  NT marks an access
// non-temporal (streamed, not kept in the caches): used for every store of
// a step (the stores of a work-item's own nodes also carry sc1, through
// WaveStores below) and for the loads whose cache lines no other lane of
// the workgroup touches (directions with e_x = 0, whose 64-lane rows are
// 512-byte aligned).  Loads shifted by one element along x share their
// boundary lines with the neighbouring wavefront and stay cached.
template <class S>
using Bits = std::conditional_t<sizeof(S) == 8, unsigned long long,
                                std::conditional_t<sizeof(S) == 4, unsigned, unsigned short>>;

template <bool NT, class S>
__device__ __forceinline__ void put(S* p, S v)
{
    if constexpr (NT) {
        __builtin_nontemporal_store(__builtin_bit_cast(Bits<S>, v), reinterpret_cast<Bits<S>*>(p));
    } else {
        *p = v;
    }
}

template <bool NT, class S>
__device__ __forceinline__ S get(const S* p)
{
    if constexpr (NT) {
        return __builtin_bit_cast(S, __builtin_nontemporal_load(reinterpret_cast<const Bits<S>*>(p)));
    } else {
        return *p;
    }
}

// Workgroups of the step kernels: 256 work-items; the occupancy bound lets
// the compiler take the VGPRs it needs to keep all Q loads of a work-item in
// flight before the collision (measured faster than forcing 8 waves per
// SIMD).
#define LBM_STEP_BOUNDS __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 8)))

// ---------------------------------------------------------------------------
// Collision at one node (Eq. (collision) with the incompressible equilibrium
// of Eq. (incompressible_feq), c_s^2 = 1/3, rho0 = 1):
//   rho = sum f,  u = sum e f + F/2,
//   feq_a = w_a (rho + 3 e_a.u + 4.5 (e_a.u)^2 - 1.5 u.u),
//   f*_a = f_a + omega (feq_a - f_a) + (1 - omega/2) w_a (3 (e_a - u).F + 9 (e_a.u)(e_a.F)).
// The update is affine in f with sum w e = 0, so it maps deviations f - w to
// deviations unchanged; the reduced-precision storages run it on f - w.
//
// COMP selects the weakly compressible equilibrium of Eq. (feq):
//   u = (sum e f + F/2)/rho,  feq_a = w_a rho (1 + 3 e_a.u + 4.5 (e_a.u)^2 - 1.5 u.u).
// On deviations (DEV) sum g = rho - 1, and feq_a - w_a =
// w_a (rho - 1 + rho (3 e_a.u + 4.5 (e_a.u)^2 - 1.5 u.u)).

template <class C>
struct CollideArgs {
    C omega;
    C F[3];
    C k3, k9;  // 3 (1 - omega/2), 9 (1 - omega/2)
};

template <int L, class C>
struct Moments {
    C rho, ux, uy, uz;  // rho: sum of the stored values (f, or f - w)
    C rf;               // density rho of the compressible model (COMP only)
};

template <int L, class C, bool FORCE, bool COMP = false, bool DEV = false>
__device__ __forceinline__ Moments<L, C> node_moments(const C (&f)[Lattice<L>::Q], const C F[3])
{
    C rho = C(-0.0), jx = C(-0.0), jy = C(-0.0), jz = C(-0.0);
    static_for<Lattice<L>::Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        rho += f[a];
        jx += eterm<kLattice<L>.e[a][0]>(f[a]);
        jy += eterm<kLattice<L>.e[a][1]>(f[a]);
        if constexpr (kDim<L> == 3) jz += eterm<kLattice<L>.e[a][2]>(f[a]);
    });
    Moments<L, C> m;
    m.rho = rho;
    if constexpr (FORCE) {
        m.ux = jx + C(0.5) * F[0];
        m.uy = jy + C(0.5) * F[1];
        m.uz = kDim<L> == 3 ? jz + C(0.5) * F[2] : C(0);
    } else {
        m.ux = jx;
        m.uy = jy;
        m.uz = kDim<L> == 3 ? jz : C(0);
    }
    m.rf = C(1);
    if constexpr (COMP) {
        m.rf = DEV ? C(1) + rho : rho;
        const C inv = C(1) / m.rf;
        m.ux *= inv;
        m.uy *= inv;
        m.uz *= inv;
    }
    return m;
}

template <int L, class C, bool FORCE, bool COMP = false, bool DEV = false>
__device__ __forceinline__ void collide(C (&f)[Lattice<L>::Q], const CollideArgs<C>& p)
{
    const Moments<L, C> m = node_moments<L, C, FORCE, COMP, DEV>(f, p.F);
    const C usq = m.ux * m.ux + m.uy * m.uy + (kDim<L> == 3 ? m.uz * m.uz : C(0));
    const C base = m.rho - C(1.5) * (COMP ? m.rf * usq : usq);
    C uF = C(0);
    if constexpr (FORCE) uF = m.ux * p.F[0] + m.uy * p.F[1] + (kDim<L> == 3 ? m.uz * p.F[2] : C(0));
    static_for<Lattice<L>::Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        constexpr int ex = kLattice<L>.e[a][0], ey = kLattice<L>.e[a][1], ez = kLattice<L>.e[a][2];
        const C w = C(kLattice<L>.w[a]);
        const C edu = eterm<ex>(m.ux) + eterm<ey>(m.uy) + eterm<ez>(m.uz);
        const C feq = w * (base + (COMP ? m.rf * edu : edu) * (C(3) + C(4.5) * edu));
        C fs = f[a] + p.omega * (feq - f[a]);
        if constexpr (FORCE) {
            const C eF = eterm<ex>(p.F[0]) + eterm<ey>(p.F[1]) + eterm<ez>(p.F[2]);
            fs += w * (p.k3 * (eF - uF) + p.k9 * edu * eF);
        }
        f[a] = fs;
    });
}

// ---------------------------------------------------------------------------
// Time-step kernels.

template <class C>
struct StepArgs {
    Dims g;
    int bx_shift;
    // Nonzero: the launch is on the grid of node_of_item_rows_on_xcd, with
    // each row's workgroups on one XCD (one-node AB steps only).
    int xcd_rows;
    CollideArgs<C> c;
};

template <class C>
__device__ __forceinline__ bool step_node(const StepArgs<C>& p, int& x, int& y, int& z)
{
    return p.xcd_rows ? node_of_item_rows_on_xcd(p.g, p.bx_shift, x, y, z) : node_of_item(p.g, p.bx_shift, x, y, z);
}

// Two FP64 populations of neighbouring nodes (x0, x0 + 1), moved as one
// 16-byte access.
typedef unsigned U32x4 __attribute__((ext_vector_type(4)));

struct Pair {
    double lo, hi;
};

// The stores of a wavefront whose work-items write their own nodes (node
// index non-decreasing with the lane), issued as buffer stores that carry
// the cache-policy bits nt | sc1 (gfx950 encoding 2 | 16): streaming, at
// device scope (sc1 without sc0), so the store goes through the XCD's L2.  Measured on MI355X, D3Q19 256^3: the
// two-node FP64 step 811 vs 830 us (+2.3 %), the one-node FP64 step 835 vs
// 862 us (+3.2 %), FP32 +1.2 %, FP16 unchanged, against non-temporal global
// stores; a plain 16-byte copy 6.69 vs 6.48 TB/s.  The buffer resource is
// wavefront-uniform: its base is the tile of the first active work-item
// (the lowest node of the wavefront), so every work-item's offset is a
// small non-negative byte count, and its record count ends at the end of
// the stored state, so a store outside it would be dropped, not written.
template <class S>
struct WaveStores {
    static constexpr int kAux = 2 | 16;  // nt | sc1
    __amdgpu_buffer_rsrc_t rs;
    size_t b0;  // element index of the resource's base

    template <int Q>
    __device__ static WaveStores make(S* dst, unsigned own, const Dims& g)
    {
        const unsigned t0 = __builtin_amdgcn_readfirstlane(own >> g.S);
        const size_t b0 = size_t(t0) * Q << g.S;
        const size_t total = (size_t((g.N + (1u << g.S) - 1) >> g.S) * Q) << g.S;
        const size_t bytes = (total - b0) * sizeof(S);
        const unsigned records = bytes > 0xFFFFFFFFull ? 0xFFFFFFFFu : unsigned(bytes);
        return {__builtin_amdgcn_make_buffer_rsrc(dst + b0, 0, records, 0x00020000), b0};
    }

    __device__ unsigned offset(size_t slot) const { return unsigned((slot - b0) * sizeof(S)); }

    __device__ void put(size_t slot, S v) const
    {
        typedef unsigned U32x2 __attribute__((ext_vector_type(2)));
        if constexpr (sizeof(S) == 8) {
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U32x2, v), rs, offset(slot), 0, kAux);
        } else if constexpr (sizeof(S) == 4) {
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rs, offset(slot), 0, kAux);
        } else {
            __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), rs, offset(slot), 0,
                                                  kAux);
        }
    }

    __device__ void put(size_t slot, Pair v) const
    {
        static_assert(sizeof(S) == 8, "pairs of FP64 populations");
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U32x4, v), rs, offset(slot), 0, kAux);
    }
};

// Fused pull-stream + bounce-back + collide (AB).
template <int L, class S, bool WALLS, bool FORCE, bool COMP, bool NT>
__global__ LBM_STEP_BOUNDS void k_step_ab(const S* __restrict__ src, S* __restrict__ dst,
                                                 StepArgs<typename Store<S>::C> p)
{
    using C = typename Store<S>::C;
    constexpr int Q = Lattice<L>::Q;
    int x, y, z;
    if (!step_node(p, x, y, z)) return;
    if (WALLS && is_solid(p.g, x, y, z)) return;
    const int TS = p.g.S;
    const unsigned own = unsigned(x) + unsigned(p.g.nx) * (unsigned(y) + unsigned(p.g.ny) * unsigned(z));
    unsigned idx[Q];
    bool wall[Q];
    link_nodes<L, WALLS, -1>(p.g, x, y, z, idx, wall);
    C f[Q];
    static_for<Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        constexpr int abar = Lattice<L>::opp(a);
        constexpr bool aligned = kLattice<L>.e[a][0] == 0;
        const S* ptr = src + ((WALLS && wall[a]) ? slot<Q>(abar, own, TS) : slot<Q>(a, idx[a], TS));
        f[a] = Store<S>::load(get<NT && aligned>(ptr));
    });
    if constexpr (WALLS) nodal_fill<L>(p.g, x, y, z, f);
    collide<L, C, FORCE, COMP, Store<S>::kDeviation>(f, p.c);
    if constexpr (NT) {
        const auto ws = WaveStores<S>::template make<Q>(dst, own, p.g);
        static_for<Q>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            ws.put(slot<Q>(a, own, TS), Store<S>::save(f[a]));
        });
    } else {
        static_for<Q>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            put<false>(dst + slot<Q>(a, own, TS), Store<S>::save(f[a]));
        });
    }
}

// Fused step (AB) of a fully periodic box whose rows each lie inside one
// tile of the stored state (nx a power of two from 64 to the tile length),
// one node per work-item.  A wavefront then covers part of one row, so the
// source row of every direction, its tile and the start of its run in that
// tile are the same for all lanes: they are computed once per wavefront in
// scalar registers, and a lane's load is that run's base plus its wrapped x
// (three values per lane), its stores the run of its own row plus x.  Same
// arithmetic per node as k_step_ab; against its per-lane 64-bit tile
// arithmetic this moves about 230 instructions per D3Q19 node from the
// vector to the scalar unit (e4m11: 840 -> 612 vector instructions), which
// pays where the step is bound by instruction issue.
template <int L, class S, bool FORCE, bool COMP, bool NT>
__global__ LBM_STEP_BOUNDS void k_step_ab_rows(const S* __restrict__ src, S* __restrict__ dst,
                                               StepArgs<typename Store<S>::C> p)
{
    using C = typename Store<S>::C;
    constexpr int Q = Lattice<L>::Q;
    const Dims& g = p.g;
    int x, y, z;
    if (!step_node(p, x, y, z)) return;  // whole wavefronts (rows of >= 64 nodes)
    y = __builtin_amdgcn_readfirstlane(y);
    z = __builtin_amdgcn_readfirstlane(z);
    const int TS = g.S;
    const unsigned mask = (1u << TS) - 1u;
    // Byte offsets of x - 1, x, x + 1 (wrapped) in a run.
    const unsigned bxm = unsigned(x == 0 ? g.nx - 1 : x - 1) * unsigned(sizeof(S));
    const unsigned bx = unsigned(x) * unsigned(sizeof(S));
    const unsigned bxp = unsigned(x == g.nx - 1 ? 0 : x + 1) * unsigned(sizeof(S));
    C f[Q];
    static_for<Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        constexpr int ex = kLattice<L>.e[a][0], ey = kLattice<L>.e[a][1], ez = kLattice<L>.e[a][2];
        int ys = y - ey;
        ys = ys < 0 ? ys + g.ny : (ys >= g.ny ? ys - g.ny : ys);
        int zs = z - ez;
        if constexpr (kDim<L> == 3) zs = zs < 0 ? zs + g.nz : (zs >= g.nz ? zs - g.nz : zs);
        else zs = z;
        // The source row's start, and the run of direction 0 there (one of
        // at most nine per wavefront, shared by the directions with the
        // same (e_y, e_z)); direction a is a << TS elements further on.
        const unsigned r = unsigned(g.nx) * (unsigned(ys) + unsigned(g.ny) * unsigned(zs));
        const char* run = reinterpret_cast<const char*>(src + (((size_t(r >> TS) * Q) << TS) | (r & mask)));
        const unsigned off = (unsigned(a) << TS) * unsigned(sizeof(S)) + (ex == 0 ? bx : (ex == 1 ? bxm : bxp));
        f[a] = Store<S>::load(get<NT && ex == 0>(reinterpret_cast<const S*>(run + off)));
    });
    collide<L, C, FORCE, COMP, Store<S>::kDeviation>(f, p.c);
    const unsigned r = unsigned(g.nx) * (unsigned(y) + unsigned(g.ny) * unsigned(z));
    S* run = dst + ((size_t(r >> TS) * Q) << TS) + (r & mask);  // own row, direction 0
    if constexpr (NT) {
        // nt | sc1 buffer stores (as WaveStores) from a resource at the run of
        // direction 0; direction a adds a << TS elements as a scalar offset.
        const size_t b0 = size_t(run - dst);
        const size_t total = (size_t((g.N + mask) >> TS) * Q) << TS;
        const size_t bytes = (total - b0) * sizeof(S);
        const unsigned records = bytes > 0xFFFFFFFFull ? 0xFFFFFFFFu : unsigned(bytes);
        const auto rs = __builtin_amdgcn_make_buffer_rsrc(run, 0, records, 0x00020000);
        const unsigned voff = unsigned(x) * unsigned(sizeof(S));
        static_for<Q>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            const unsigned soff = (unsigned(a) << TS) * unsigned(sizeof(S));
            const S v = Store<S>::save(f[a]);
            if constexpr (sizeof(S) == 8) {
                typedef unsigned U32x2 __attribute__((ext_vector_type(2)));
                __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U32x2, v), rs, voff, soff,
                                                      WaveStores<S>::kAux);
            } else if constexpr (sizeof(S) == 4) {
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rs, voff, soff,
                                                      WaveStores<S>::kAux);
            } else {
                __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), rs, voff, soff,
                                                      WaveStores<S>::kAux);
            }
        });
    } else {
        static_for<Q>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            put<false>(run + (size_t(a) << TS) + unsigned(x), Store<S>::save(f[a]));
        });
    }
}

// Fused step of a fully periodic FP64 box with two nodes per work-item
// (AB).  A work-item owns nodes (x0, x0 + 1), x0 even, and reads every
// direction as one aligned 16-byte load of the source row at (x0, x0 + 1);
// a direction with e_x = +1 needs (x0 - 1, x0), so the element x0 - 1 comes
// from the neighbouring lane by a wave shift (DPP wave_shr:1, a GFX9-family
// control that gfx950 keeps), and symmetrically e_x = -1 takes x0 + 2 from
// the next lane (wave_shl:1).  The lane at a wavefront edge or a row end
// reads that one element itself (periodic wrap).  Same arithmetic per node
// as k_step_ab; 16-byte accesses measured 3 % faster for FP64 storage on
// large boxes.  Needs an even nx; lanes per row BXL = 1 << bxl_shift.
template <bool NT>
__device__ __forceinline__ Pair get_pair(const double* p)
{
    const U32x4* q = reinterpret_cast<const U32x4*>(p);
    if constexpr (NT) return __builtin_bit_cast(Pair, __builtin_nontemporal_load(q));
    else return __builtin_bit_cast(Pair, *q);
}

__device__ __forceinline__ void put_pair(double* p, Pair v)
{
    __builtin_nontemporal_store(__builtin_bit_cast(U32x4, v), reinterpret_cast<U32x4*>(p));
}


// Lane i receives v of lane i - 1 (SHIFT = 0x138, wave_shr:1) or of lane
// i + 1 (SHIFT = 0x130, wave_shl:1); the edge lane keeps its own v.
template <int SHIFT>
__device__ __forceinline__ double wave_shift(double v)
{
    int2 w = __builtin_bit_cast(int2, v);
    w.x = __builtin_amdgcn_update_dpp(w.x, w.x, SHIFT, 0xf, 0xf, false);
    w.y = __builtin_amdgcn_update_dpp(w.y, w.y, SHIFT, 0xf, 0xf, false);
    return __builtin_bit_cast(double, w);
}

template <int L, bool FORCE, bool COMP, bool NT>
__global__ LBM_STEP_BOUNDS void k_step_ab_pairs(const double* __restrict__ src,
                                                double* __restrict__ dst, StepArgs<double> p,
                                                int bxl_shift)
{
    constexpr int Q = Lattice<L>::Q;
    const Dims& g = p.g;
    const int lane = threadIdx.x & 63;
    const int x0 = ((blockIdx.x << bxl_shift) + int(threadIdx.x & ((1u << bxl_shift) - 1u))) * 2;
    const int y = blockIdx.y * (256 >> bxl_shift) + int(threadIdx.x >> bxl_shift);
    const int z = blockIdx.z;
    // Idle work-items (past the row or the last row) still take part in the
    // wave shifts; they read row 0 and store nothing.
    const bool active = x0 < g.nx && y < g.ny;
    const int xa = active ? x0 : 0, ya = active ? y : 0;
    const int TS = g.S;
    double f0[Q], f1[Q];
    static_for<Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        constexpr int ex = kLattice<L>.e[a][0], ey = kLattice<L>.e[a][1], ez = kLattice<L>.e[a][2];
        int ys = ya - ey;
        ys = ys < 0 ? ys + g.ny : (ys >= g.ny ? ys - g.ny : ys);
        int zs = z - ez;
        if constexpr (kDim<L> == 3) zs = zs < 0 ? zs + g.nz : (zs >= g.nz ? zs - g.nz : zs);
        else zs = z;
        const unsigned row = unsigned(g.nx) * (unsigned(ys) + unsigned(g.ny) * unsigned(zs));
        const Pair v = get_pair<NT && ex == 0>(src + slot<Q>(a, row + unsigned(xa), TS));
        if constexpr (ex == 0) {
            f0[a] = v.lo;
            f1[a] = v.hi;
        } else if constexpr (ex == 1) {  // sources x0 - 1, x0
            double first = wave_shift<0x138>(v.hi);
            if (lane == 0 || xa == 0) first = src[slot<Q>(a, row + unsigned(xa == 0 ? g.nx - 1 : xa - 1), TS)];
            f0[a] = first;
            f1[a] = v.lo;
        } else {  // sources x0 + 1, x0 + 2
            double last = wave_shift<0x130>(v.lo);
            if (lane == 63 || xa + 2 >= g.nx) last = src[slot<Q>(a, row + unsigned(xa + 2 >= g.nx ? 0 : xa + 2), TS)];
            f0[a] = v.hi;
            f1[a] = last;
        }
    });
    if (!active) return;
    collide<L, double, FORCE, COMP, false>(f0, p.c);
    collide<L, double, FORCE, COMP, false>(f1, p.c);
    const unsigned own = unsigned(x0) + unsigned(g.nx) * (unsigned(y) + unsigned(g.ny) * unsigned(z));
    const auto ws = WaveStores<double>::make<Q>(dst, own, g);
    static_for<Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        ws.put(slot<Q>(a, own, TS), Pair{f0[a], f1[a]});
    });
}

// AA steps of a periodic FP64 box with two nodes per work-item (see
// k_step_ab_pairs for the layout of work-items and the wave shifts).  The
// even step reads and writes the work-item's own aligned node pairs only.
// The odd step reads the x-shifted source pairs like k_step_ab_pairs and
// writes f*_a to the slots it read for abar, which are x-shifted the other
// way: the aligned destination pair (x0, x0 + 1) takes one value from this
// work-item and one from its neighbour lane.  A work-item at a wavefront
// edge or a row end writes its outer value as a single element and the
// work-item across the edge leaves that element alone, so every address is
// read and written by one work-item, as the in-place update needs.  Those
// single elements go through the cache (not non-temporal): their lines are
// completed by the neighbouring wavefront's stores and then leave L2 as
// whole lines (with non-temporal edge stores 2 % more bytes reached HBM and
// the odd step ran 5 % slower on MI355X).
template <int L, bool FORCE, bool COMP, bool NT>
__global__ LBM_STEP_BOUNDS void k_step_aa_even_pairs(double* __restrict__ A, StepArgs<double> p,
                                                     int bxl_shift)
{
    constexpr int Q = Lattice<L>::Q;
    const Dims& g = p.g;
    const int x0 = ((blockIdx.x << bxl_shift) + int(threadIdx.x & ((1u << bxl_shift) - 1u))) * 2;
    const int y = blockIdx.y * (256 >> bxl_shift) + int(threadIdx.x >> bxl_shift);
    const int z = blockIdx.z;
    if (x0 >= g.nx || y >= g.ny) return;
    const int TS = g.S;
    const unsigned own = unsigned(x0) + unsigned(g.nx) * (unsigned(y) + unsigned(g.ny) * unsigned(z));
    double f0[Q], f1[Q];
    static_for<Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        const Pair v = get_pair<NT>(A + slot<Q>(a, own, TS));
        f0[a] = v.lo;
        f1[a] = v.hi;
    });
    collide<L, double, FORCE, COMP, false>(f0, p.c);
    collide<L, double, FORCE, COMP, false>(f1, p.c);
    const auto ws = WaveStores<double>::make<Q>(A, own, g);
    static_for<Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        ws.put(slot<Q>(Lattice<L>::opp(a), own, TS), Pair{f0[a], f1[a]});
    });
}

template <int L, bool FORCE, bool COMP, bool NT>
__global__ LBM_STEP_BOUNDS void k_step_aa_odd_pairs(double* __restrict__ A, StepArgs<double> p,
                                                    int bxl_shift)
{
    constexpr int Q = Lattice<L>::Q;
    const Dims& g = p.g;
    const int lane = threadIdx.x & 63;
    const int x0 = ((blockIdx.x << bxl_shift) + int(threadIdx.x & ((1u << bxl_shift) - 1u))) * 2;
    const int y = blockIdx.y * (256 >> bxl_shift) + int(threadIdx.x >> bxl_shift);
    const int z = blockIdx.z;
    // Idle work-items take part in the wave shifts, read row 0 and write
    // nothing.
    const bool active = x0 < g.nx && y < g.ny;
    const int xa = active ? x0 : 0, ya = active ? y : 0;
    const bool left_edge = lane == 0 || xa == 0;        // x0 - 1 is across an edge
    const bool right_edge = lane == 63 || xa + 2 >= g.nx;  // x0 + 2 is across an edge
    const int xl = xa == 0 ? g.nx - 1 : xa - 1;            // x0 - 1, wrapped
    const int xr = xa + 2 >= g.nx ? 0 : xa + 2;            // x0 + 2, wrapped
    const int TS = g.S;
    unsigned row[Q];  // the row of x - e_a, where f_a(x) is read and f*_abar(x) written
    double f0[Q], f1[Q];
    static_for<Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        constexpr int ex = kLattice<L>.e[a][0], ey = kLattice<L>.e[a][1], ez = kLattice<L>.e[a][2];
        int ys = ya - ey;
        ys = ys < 0 ? ys + g.ny : (ys >= g.ny ? ys - g.ny : ys);
        int zs = z - ez;
        if constexpr (kDim<L> == 3) zs = zs < 0 ? zs + g.nz : (zs >= g.nz ? zs - g.nz : zs);
        else zs = z;
        row[a] = unsigned(g.nx) * (unsigned(ys) + unsigned(g.ny) * unsigned(zs));
        constexpr int abar = Lattice<L>::opp(a);
        const Pair v = get_pair<NT && ex == 0>(A + slot<Q>(abar, row[a] + unsigned(xa), TS));
        if constexpr (ex == 0) {
            f0[a] = v.lo;
            f1[a] = v.hi;
        } else if constexpr (ex == 1) {  // sources x0 - 1, x0
            double first = wave_shift<0x138>(v.hi);
            if (left_edge) first = A[slot<Q>(abar, row[a] + unsigned(xl), TS)];
            f0[a] = first;
            f1[a] = v.lo;
        } else {  // sources x0 + 1, x0 + 2
            double last = wave_shift<0x130>(v.lo);
            if (right_edge) last = A[slot<Q>(abar, row[a] + unsigned(xr), TS)];
            f0[a] = v.hi;
            f1[a] = last;
        }
    });
    collide<L, double, FORCE, COMP, false>(f0, p.c);
    collide<L, double, FORCE, COMP, false>(f1, p.c);
    // f*_a(x) goes to slot a of x + e_a, in the row read for abar.
    static_for<Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        constexpr int ex = kLattice<L>.e[a][0];
        constexpr int abar = Lattice<L>::opp(a);
        if constexpr (ex == 0) {
            if (active) put_pair(A + slot<Q>(a, row[abar] + unsigned(x0), TS), Pair{f0[a], f1[a]});
        } else if constexpr (ex == 1) {  // destinations x0 + 1, x0 + 2
            const double from_left = wave_shift<0x138>(f1[a]);  // f*_a(x0 - 1) -> x0
            if (active) {
                if (left_edge) put<false>(A + slot<Q>(a, row[abar] + unsigned(x0 + 1), TS), f0[a]);
                else put_pair(A + slot<Q>(a, row[abar] + unsigned(x0), TS), Pair{from_left, f0[a]});
                if (right_edge) put<false>(A + slot<Q>(a, row[abar] + unsigned(xr), TS), f1[a]);
            }
        } else {  // destinations x0 - 1, x0
            const double from_right = wave_shift<0x130>(f0[a]);  // f*_a(x0 + 2) -> x0 + 1
            if (active) {
                if (right_edge) put<false>(A + slot<Q>(a, row[abar] + unsigned(x0), TS), f1[a]);
                else put_pair(A + slot<Q>(a, row[abar] + unsigned(x0), TS), Pair{f1[a], from_right});
                if (left_edge) put<false>(A + slot<Q>(a, row[abar] + unsigned(xl), TS), f0[a]);
            }
        }
    });
}

// AA even step: own slots in, opposite own slots out.
template <int L, class S, bool WALLS, bool FORCE, bool COMP, bool NT>
__global__ LBM_STEP_BOUNDS void k_step_aa_even(S* __restrict__ A,
                                                      StepArgs<typename Store<S>::C> p)
{
    using C = typename Store<S>::C;
    constexpr int Q = Lattice<L>::Q;
    int x, y, z;
    if (!node_of_item(p.g, p.bx_shift, x, y, z)) return;
    if (WALLS && is_solid(p.g, x, y, z)) return;
    const int TS = p.g.S;
    const unsigned own = unsigned(x) + unsigned(p.g.nx) * (unsigned(y) + unsigned(p.g.ny) * unsigned(z));
    C f[Q];
    static_for<Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        f[a] = Store<S>::load(get<NT>(A + slot<Q>(a, own, TS)));
    });
    if constexpr (WALLS) nodal_fill<L>(p.g, x, y, z, f);
    collide<L, C, FORCE, COMP, Store<S>::kDeviation>(f, p.c);
    if constexpr (NT) {
        const auto ws = WaveStores<S>::template make<Q>(A, own, p.g);
        static_for<Q>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            ws.put(slot<Q>(Lattice<L>::opp(a), own, TS), Store<S>::save(f[a]));
        });
    } else {
        static_for<Q>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            put<false>(A + slot<Q>(Lattice<L>::opp(a), own, TS), Store<S>::save(f[a]));
        });
    }
}

// AA odd step: f_a(x) from slot abar of x - e_a (or slot a of x at a wall);
// f*_a(x) goes to slot a of x + e_a (or slot abar of x at a wall), which is
// the address read for direction abar.
template <int L, class S, bool WALLS, bool FORCE, bool COMP, bool NT>
__global__ LBM_STEP_BOUNDS void k_step_aa_odd(S* __restrict__ A,
                                                     StepArgs<typename Store<S>::C> p)
{
    using C = typename Store<S>::C;
    constexpr int Q = Lattice<L>::Q;
    int x, y, z;
    if (!node_of_item(p.g, p.bx_shift, x, y, z)) return;
    if (WALLS && is_solid(p.g, x, y, z)) return;
    const int TS = p.g.S;
    const unsigned own = unsigned(x) + unsigned(p.g.nx) * (unsigned(y) + unsigned(p.g.ny) * unsigned(z));
    unsigned idx[Q];
    bool wall[Q];
    link_nodes<L, WALLS, -1>(p.g, x, y, z, idx, wall);
    size_t off[Q];
    static_for<Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        constexpr int abar = Lattice<L>::opp(a);
        off[a] = (WALLS && wall[a]) ? slot<Q>(a, own, TS) : slot<Q>(abar, idx[a], TS);
    });
    C f[Q];
    static_for<Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        f[a] = Store<S>::load(get<NT && kLattice<L>.e[a][0] == 0>(A + off[a]));
    });
    if constexpr (WALLS) nodal_fill<L>(p.g, x, y, z, f);
    collide<L, C, FORCE, COMP, Store<S>::kDeviation>(f, p.c);
    static_for<Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        put<NT>(A + off[Lattice<L>::opp(a)], Store<S>::save(f[a]));
    });
}

// ---------------------------------------------------------------------------
// State import / export and moments.  These run on set-up and monitor steps
// only; they take the canonical FP64 f^n ([Q][N]) through the bijection of
// gather_offset.

struct IoArgs {
    Dims g;
    int bx_shift;
    int mode;  // GatherMode of the stored state
    int comp;  // compressible model: u = (sum e f + F/2)/rho
    double F[3];
};

// f^n from equilibrium (rho, u) plus optional noise, or from f (when f is
// non-null), written into the stored state.  Deviation storages store f - w.
template <int L, class S, bool WALLS>
__global__ __launch_bounds__(256) void k_import(S* __restrict__ A, const double* __restrict__ f,
                                                const double* __restrict__ rho,
                                                const double* __restrict__ u,
                                                const double* __restrict__ noise, IoArgs p)
{
    constexpr int Q = Lattice<L>::Q;
    int x, y, z;
    if (!node_of_item(p.g, p.bx_shift, x, y, z)) return;
    const unsigned N = p.g.N;
    const unsigned own = unsigned(x) + unsigned(p.g.nx) * (unsigned(y) + unsigned(p.g.ny) * unsigned(z));
    if (WALLS && is_solid(p.g, x, y, z)) return;
    unsigned idx[Q];
    bool wall[Q];
    link_nodes<L, WALLS, -1>(p.g, x, y, z, idx, wall);
    double fn[Q];
    if (f) {
        static_for<Q>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            fn[a] = f[size_t(a) * N + own];
        });
    } else {
        const double r = rho[own];
        const double ux = u[own], uy = u[size_t(N) + own], uz = kDim<L> == 3 ? u[2 * size_t(N) + own] : 0.0;
        const double usq = ux * ux + uy * uy + uz * uz;
        static_for<Q>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            constexpr auto& LT = kLattice<L>;
            const double edu = eterm<LT.e[a][0]>(ux) + eterm<LT.e[a][1]>(uy) + eterm<LT.e[a][2]>(uz);
            const double rq = p.comp ? r : 1.0;
            double v = LT.w[a] * (r + rq * (3.0 * edu + 4.5 * edu * edu - 1.5 * usq));
            if (noise) v += noise[size_t(a) * N + own];
            fn[a] = v;
        });
    }
    static_for<Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        double v = fn[a];
        if constexpr (Store<S>::kDeviation) v -= kLattice<L>.w[a];
        A[gather_offset<L>(p.mode, a, own, idx[a], WALLS && wall[a], p.g.S)] =
            Store<S>::save(typename Store<S>::C(v));
    });
}

// Gathers f^n (in the storage's arithmetic type, as stored: f or f - w),
// with Eq. (bb) applied on nodal wall nodes.
template <int L, class S, bool WALLS>
__device__ __forceinline__ void gather_node(const S* __restrict__ A, const IoArgs& p, int x, int y,
                                            int z, unsigned own,
                                            typename Store<S>::C (&f)[Lattice<L>::Q])
{
    constexpr int Q = Lattice<L>::Q;
    unsigned idx[Q];
    bool wall[Q];
    link_nodes<L, WALLS, -1>(p.g, x, y, z, idx, wall);
    static_for<Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        f[a] = Store<S>::load(A[gather_offset<L>(p.mode, a, own, idx[a], WALLS && wall[a], p.g.S)]);
    });
    if constexpr (WALLS) nodal_fill<L>(p.g, x, y, z, f);
}

// rho, u of f^n as the model defines them, and the sum of the stored values
// (rho, or rho - 1 for deviation storage), in FP64.
template <int L, class S>
__device__ __forceinline__ void node_rho_u(const typename Store<S>::C (&fn)[Lattice<L>::Q],
                                           const IoArgs& p, double& sum, double& rho,
                                           double (&u)[3])
{
    using C = typename Store<S>::C;
    const C F[3] = {C(p.F[0]), C(p.F[1]), C(p.F[2])};
    const Moments<L, C> m = node_moments<L, C, true>(fn, F);
    sum = double(m.rho);
    rho = Store<S>::kDeviation ? 1.0 + double(m.rho) : double(m.rho);
    u[0] = double(m.ux);
    u[1] = double(m.uy);
    u[2] = double(m.uz);
    if (p.comp) {
        // u = (j + F/2)/rho in the arithmetic type, as the collision forms it
        const C inv = C(1) / C(Store<S>::kDeviation ? C(1) + m.rho : m.rho);
        u[0] = double(m.ux * inv);
        u[1] = double(m.uy * inv);
        u[2] = double(m.uz * inv);
    }
}

template <int L, class S, bool WALLS>
__global__ __launch_bounds__(256) void k_export(const S* __restrict__ A, double* __restrict__ f,
                                                IoArgs p)
{
    constexpr int Q = Lattice<L>::Q;
    int x, y, z;
    if (!node_of_item(p.g, p.bx_shift, x, y, z)) return;
    const unsigned N = p.g.N;
    const unsigned own = unsigned(x) + unsigned(p.g.nx) * (unsigned(y) + unsigned(p.g.ny) * unsigned(z));
    if (WALLS && is_solid(p.g, x, y, z)) {
        for (int a = 0; a < Q; ++a) f[size_t(a) * N + own] = 0.0;
        return;
    }
    typename Store<S>::C fn[Q];
    gather_node<L, S, WALLS>(A, p, x, y, z, own, fn);
    static_for<Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        double v = double(fn[a]);
        if constexpr (Store<S>::kDeviation) v += kLattice<L>.w[a];
        f[size_t(a) * N + own] = v;
    });
}

// PostProcessing: rho = sum f (= 1 + sum (f - w) for deviation storage),
// u = sum e f + F/2 (divided by rho in the compressible model).
template <int L, class S, bool WALLS, class O>
__global__ __launch_bounds__(256) void k_moments(const S* __restrict__ A, O* __restrict__ rho,
                                                 O* __restrict__ u, IoArgs p)
{
    using C = typename Store<S>::C;
    constexpr int Q = Lattice<L>::Q;
    int x, y, z;
    if (!node_of_item(p.g, p.bx_shift, x, y, z)) return;
    const unsigned N = p.g.N;
    const unsigned own = unsigned(x) + unsigned(p.g.nx) * (unsigned(y) + unsigned(p.g.ny) * unsigned(z));
    if (WALLS && is_solid(p.g, x, y, z)) {
        if (rho) rho[own] = O(0);
        if (u) u[own] = u[size_t(N) + own] = u[2 * size_t(N) + own] = O(0);
        return;
    }
    C fn[Q];
    gather_node<L, S, WALLS>(A, p, x, y, z, own, fn);
    double sum, r, v[3];
    node_rho_u<L, S>(fn, p, sum, r, v);
    if (rho) rho[own] = O(r);
    if (u) {
        u[own] = O(v[0]);
        u[size_t(N) + own] = O(v[1]);
        u[2 * size_t(N) + own] = O(v[2]);
    }
}

// Monitor: per-block FP64 partials (sum rho - rho_ref, sum rho_m |u|^2,
// max |u|, non-finite count; rho_m = 1 in the incompressible model, rho in
// the compressible one) over a fixed grid-stride assignment and a fixed
// in-block tree, so the result is independent of scheduling.
constexpr int kReduceThreads = 256;
constexpr int kReduceBlocks = 1024;

template <int L, class S, bool WALLS>
__global__ __launch_bounds__(kReduceThreads) void k_reduce_partials(const S* __restrict__ A,
                                                                    double* __restrict__ partials,
                                                                    IoArgs p)
{
    using C = typename Store<S>::C;
    constexpr int Q = Lattice<L>::Q;
    __shared__ double s_mass[kReduceThreads], s_ke[kReduceThreads], s_max[kReduceThreads],
        s_bad[kReduceThreads], s_cnt[kReduceThreads];
    double mass = 0.0, ke = 0.0, umax = 0.0, bad = 0.0, cnt = 0.0;
    const unsigned N = p.g.N;
    for (unsigned n = blockIdx.x * kReduceThreads + threadIdx.x; n < N;
         n += kReduceBlocks * kReduceThreads) {
        const int x = int(n % unsigned(p.g.nx));
        const unsigned yz = n / unsigned(p.g.nx);
        const int y = int(yz % unsigned(p.g.ny));
        const int z = int(yz / unsigned(p.g.ny));
        if (WALLS && is_solid(p.g, x, y, z)) continue;
        C fn[Q];
        gather_node<L, S, WALLS>(A, p, x, y, z, n, fn);
        for (int a = 0; a < Q; ++a)
            if (!isfinite(double(fn[a]))) bad += 1.0;
        double sum, r, v[3];
        node_rho_u<L, S>(fn, p, sum, r, v);
        const double u2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        mass += sum;
        ke += p.comp ? r * u2 : u2;
        umax = fmax(umax, sqrt(u2));
        cnt += 1.0;
    }
    const int t = threadIdx.x;
    s_mass[t] = mass;
    s_ke[t] = ke;
    s_max[t] = umax;
    s_bad[t] = bad;
    s_cnt[t] = cnt;
    __syncthreads();
    for (int h = kReduceThreads / 2; h > 0; h >>= 1) {
        if (t < h) {
            s_mass[t] += s_mass[t + h];
            s_ke[t] += s_ke[t + h];
            s_max[t] = fmax(s_max[t], s_max[t + h]);
            s_bad[t] += s_bad[t + h];
            s_cnt[t] += s_cnt[t + h];
        }
        __syncthreads();
    }
    if (t == 0) {
        double* o = partials + 5 * size_t(blockIdx.x);
        o[0] = s_mass[0];
        o[1] = s_ke[0];
        o[2] = s_max[0];
        o[3] = s_bad[0];
        o[4] = s_cnt[0];
    }
}

// Sums the block partials in block order with one block; out[0..3] = mass
// (plus the fluid-node count for deviation storage), kinetic energy
// (1/2) sum rho_m |u|^2, max |u|, non-finite count.
[[maybe_unused]] static __global__ __launch_bounds__(kReduceThreads) void k_reduce_final(const double* __restrict__ partials,
                                                                 int nblocks, int deviation,
                                                                 double* __restrict__ out)
{
    __shared__ double s[5][kReduceThreads];
    const int t = threadIdx.x;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = t; b < nblocks; b += kReduceThreads) {
        const double* o = partials + 5 * size_t(b);
        acc[0] += o[0];
        acc[1] += o[1];
        acc[2] = fmax(acc[2], o[2]);
        acc[3] += o[3];
        acc[4] += o[4];
    }
    for (int k = 0; k < 5; ++k) s[k][t] = acc[k];
    __syncthreads();
    for (int h = kReduceThreads / 2; h > 0; h >>= 1) {
        if (t < h) {
            s[0][t] += s[0][t + h];
            s[1][t] += s[1][t + h];
            s[2][t] = fmax(s[2][t], s[2][t + h]);
            s[3][t] += s[3][t + h];
            s[4][t] += s[4][t + h];
        }
        __syncthreads();
    }
    if (t == 0) {
        out[0] = deviation ? s[0][0] + s[4][0] : s[0][0];
        out[1] = 0.5 * s[1][0];
        out[2] = s[2][0];
        out[3] = s[3][0];
    }
}

// Sums slots 0..2 of the block partials in block order (one workgroup).
[[maybe_unused]] static __global__ __launch_bounds__(kReduceThreads) void k_sum3(const double* __restrict__ partials,
                                                         int nblocks, double* __restrict__ out)
{
    __shared__ double s[3][kReduceThreads];
    const int t = threadIdx.x;
    double v[3] = {0.0, 0.0, 0.0};
    for (int b = t; b < nblocks; b += kReduceThreads)
        for (int d = 0; d < 3; ++d) v[d] += partials[5 * size_t(b) + d];
    for (int d = 0; d < 3; ++d) s[d][t] = v[d];
    __syncthreads();
    for (int h = kReduceThreads / 2; h > 0; h >>= 1) {
        if (t < h)
            for (int d = 0; d < 3; ++d) s[d][t] += s[d][t + h];
        __syncthreads();
    }
    if (t == 0)
        for (int d = 0; d < 3; ++d) out[d] = s[d][0];
}

// ---------------------------------------------------------------------------
// Solid mask (SetGeometry with a user geo array) and wall force.

// Link bits of every node from a solid mask (nonzero = solid) and the axis
// boundaries; g.links must be null here.
template <int L>
__global__ __launch_bounds__(256) void k_build_links(const unsigned char* __restrict__ mask,
                                                     unsigned* __restrict__ links, Dims g,
                                                     int bx_shift)
{
    constexpr int Q = Lattice<L>::Q;
    int x, y, z;
    if (!node_of_item(g, bx_shift, x, y, z)) return;
    const unsigned own = node_index(g, x, y, z);
    unsigned idx[Q];
    bool wall[Q];
    link_nodes<L, true, -1>(g, x, y, z, idx, wall);
    unsigned bits = (axis_solid(g, x, y, z) || mask[own]) ? (1u << 31) : 0u;
    static_for<Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        if (wall[a] || mask[idx[a]]) bits |= 1u << a;
    });
    links[own] = bits;
}

// Momentum exchanged with the walls in the last propagation (the drag
// evaluation of Sec. 4): for each fluid node x and direction a whose
// neighbour x + e_a is a wall, the population that left along a came back
// as f^n_abar(x), so the wall received 2 f^n_abar(x) e_a.  Links that cross
// a wall of the nodal scheme are not counted.  Per-block FP64 partials over
// a fixed grid-stride assignment (slots 0..2 of 5).
template <int L, class S>
__global__ __launch_bounds__(kReduceThreads) void k_wall_force(const S* __restrict__ A,
                                                               double* __restrict__ partials,
                                                               IoArgs p)
{
    using C = typename Store<S>::C;
    constexpr int Q = Lattice<L>::Q;
    __shared__ double s[3][kReduceThreads];
    double F[3] = {0.0, 0.0, 0.0};
    const unsigned N = p.g.N;
    for (unsigned n = blockIdx.x * kReduceThreads + threadIdx.x; n < N;
         n += kReduceBlocks * kReduceThreads) {
        const int x = int(n % unsigned(p.g.nx));
        const unsigned yz = n / unsigned(p.g.nx);
        const int y = int(yz % unsigned(p.g.ny));
        const int z = int(yz / unsigned(p.g.ny));
        if (is_solid(p.g, x, y, z)) continue;
        unsigned idx[Q];
        bool out[Q];
        link_nodes<L, true, +1>(p.g, x, y, z, idx, out);
        for (int a = 0; a < Q; ++a) out[a] = out[a] && !beyond_nodal<L, +1>(p.g, x, y, z, a);
        bool any = false;
        for (int a = 0; a < Q; ++a) any = any || out[a];
        if (!any) continue;
        C fn[Q];
        gather_node<L, S, true>(A, p, x, y, z, n, fn);
        static_for<Q>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            constexpr int abar = Lattice<L>::opp(a);
            if (out[a]) {
                double f = double(fn[abar]);
                if constexpr (Store<S>::kDeviation) f += kLattice<L>.w[abar];
                F[0] += eterm<kLattice<L>.e[a][0]>(2.0 * f);
                F[1] += eterm<kLattice<L>.e[a][1]>(2.0 * f);
                F[2] += eterm<kLattice<L>.e[a][2]>(2.0 * f);
            }
        });
    }
    const int t = threadIdx.x;
    for (int d = 0; d < 3; ++d) s[d][t] = F[d];
    __syncthreads();
    for (int h = kReduceThreads / 2; h > 0; h >>= 1) {
        if (t < h)
            for (int d = 0; d < 3; ++d) s[d][t] += s[d][t + h];
        __syncthreads();
    }
    if (t == 0) {
        double* o = partials + 5 * size_t(blockIdx.x);
        o[0] = s[0][0];
        o[1] = s[1][0];
        o[2] = s[2][0];
        o[3] = 0.0;
        o[4] = 0.0;
    }
}

}  // namespace imexlbm
