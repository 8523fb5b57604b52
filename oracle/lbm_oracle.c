/*
 * CPU oracle of the IMEXLBM time step (Liu, Patel, Balakrishnan, Lee,
 * "IMEXLBM 1.0", 2022): a plain, slow, FP64 restatement of the method that
 * the GPU path is checked against.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or constant with the HIP library.
 *
 * Layout follows the paper (Sec. 3.3, Table 3): populations are AoS,
 * f[id*Q + a], with id = x + nx*(y + ny*z) (unit stride in x, strides dy and
 * dz); f holds the post-propagation populations and fb the post-collision
 * "backup" copy; rho (= p/c_s^2) and u are the PostProcessing fields.
 * Inputs and outputs cross this API in the canonical structure-of-arrays
 * order [component][z][y][x].
 *
 * One time step follows the main loop of Sec. 3.1: Collision (Eq.
 * (collision)), BoundaryCondition (bounce-back, Eq. (bb), a pre-propagation
 * condition), Propagation (Eq. (propagation)) and PostProcessing (moments).
 *
 * Built with -ffp-contract=off: every product and sum is rounded as written.
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define ORC_QMAX 27
#define ORC_RHO0 1.0 /* constant density of the incompressible model (Table 3) */

typedef struct {
    int Q, D;
    int e[ORC_QMAX][3];
    double t[ORC_QMAX];
} orc_lattice;

/* D2Q9 velocities and weights exactly as printed in Sec. 2.1 (c = 1). */
static const int D2Q9_EX[9] = {-1, -1, -1, 0, 0, 0, 1, 1, 1};
static const int D2Q9_EY[9] = {-1, 0, 1, -1, 0, 1, -1, 0, 1};
static const double D2Q9_T[9] = {1.0 / 36, 1.0 / 9, 1.0 / 36, 1.0 / 9, 4.0 / 9,
                                 1.0 / 9, 1.0 / 36, 1.0 / 9, 1.0 / 36};

/*
 * D3Q19 (Qian et al.; the numbering figure of Sec. 2.1 is not reproduced in
 * the text).  Reading: the D2Q9 rule of Sec. 2.1 extended to three
 * dimensions -- lexicographic in (e_x, e_y, e_z) with e_x slowest, corners
 * (|e_x|+|e_y|+|e_z| = 3) removed -- so the opposite of a is 18 - a as the
 * paper requires.  Weights: rest 1/3, the 6 faces 1/18, the 12 edges 1/36.
 */
static const int D3Q19_E[19][3] = {
    {-1, -1, 0}, {-1, 0, -1}, {-1, 0, 0}, {-1, 0, 1}, {-1, 1, 0},
    {0, -1, -1}, {0, -1, 0},  {0, -1, 1}, {0, 0, -1}, {0, 0, 0},
    {0, 0, 1},   {0, 1, -1},  {0, 1, 0},  {0, 1, 1},  {1, -1, 0},
    {1, 0, -1},  {1, 0, 0},   {1, 0, 1},  {1, 1, 0}};
static const double D3Q19_T[19] = {
    1.0 / 36, 1.0 / 36, 1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 18,
    1.0 / 36, 1.0 / 18, 1.0 / 3,  1.0 / 18, 1.0 / 36, 1.0 / 18, 1.0 / 36,
    1.0 / 36, 1.0 / 36, 1.0 / 18, 1.0 / 36, 1.0 / 36};

/*
 * D3Q27 (the paper's validation lattice, Sec. 5): all of {-1,0,1}^3 in the
 * same lexicographic order (e_x slowest), so the opposite of a is 26 - a.
 * Weights: rest 8/27, faces 2/27, edges 1/54, corners 1/216.
 */
static const int D3Q27_E[27][3] = {
    {-1, -1, -1}, {-1, -1, 0}, {-1, -1, 1}, {-1, 0, -1}, {-1, 0, 0}, {-1, 0, 1},
    {-1, 1, -1},  {-1, 1, 0},  {-1, 1, 1},  {0, -1, -1}, {0, -1, 0}, {0, -1, 1},
    {0, 0, -1},   {0, 0, 0},   {0, 0, 1},   {0, 1, -1},  {0, 1, 0},  {0, 1, 1},
    {1, -1, -1},  {1, -1, 0},  {1, -1, 1},  {1, 0, -1},  {1, 0, 0},  {1, 0, 1},
    {1, 1, -1},   {1, 1, 0},   {1, 1, 1}};
static const double D3Q27_T[27] = {
    1.0 / 216, 1.0 / 54, 1.0 / 216, 1.0 / 54, 2.0 / 27, 1.0 / 54, 1.0 / 216, 1.0 / 54, 1.0 / 216,
    1.0 / 54,  2.0 / 27, 1.0 / 54,  2.0 / 27, 8.0 / 27, 2.0 / 27, 1.0 / 54,  2.0 / 27, 1.0 / 54,
    1.0 / 216, 1.0 / 54, 1.0 / 216, 1.0 / 54, 2.0 / 27, 1.0 / 54, 1.0 / 216, 1.0 / 54, 1.0 / 216};

static int make_lattice(int lattice, orc_lattice* L)
{
    memset(L, 0, sizeof(*L));
    if (lattice == ORC_D2Q9) {
        L->Q = 9;
        L->D = 2;
        for (int a = 0; a < 9; ++a) {
            L->e[a][0] = D2Q9_EX[a];
            L->e[a][1] = D2Q9_EY[a];
            L->e[a][2] = 0;
            L->t[a] = D2Q9_T[a];
        }
        return 0;
    }
    if (lattice == ORC_D3Q19) {
        L->Q = 19;
        L->D = 3;
        for (int a = 0; a < 19; ++a) {
            for (int d = 0; d < 3; ++d) L->e[a][d] = D3Q19_E[a][d];
            L->t[a] = D3Q19_T[a];
        }
        return 0;
    }
    if (lattice == ORC_D3Q27) {
        L->Q = 27;
        L->D = 3;
        for (int a = 0; a < 27; ++a) {
            for (int d = 0; d < 3; ++d) L->e[a][d] = D3Q27_E[a][d];
            L->t[a] = D3Q27_T[a];
        }
        return 0;
    }
    return ORC_EINVAL;
}

/* The opposite direction, abar = m - 1 - a (Sec. 2.1). */
static int opposite(const orc_lattice* L, int a) { return L->Q - 1 - a; }

#define T double
#define SFX r
#include "node.inc"
#undef T
#undef SFX

#define T double complex
#define SFX c
#include "node.inc"
#undef T
#undef SFX

/* Neumaier's compensated summation. */
typedef struct {
    double sum, comp;
} kahan;
static void kahan_add(kahan* k, double v)
{
    double t = k->sum + v;
    if (fabs(k->sum) >= fabs(v))
        k->comp += (k->sum - t) + v;
    else
        k->comp += (v - t) + k->sum;
    k->sum = t;
}

struct orc_sim {
    orc_lattice L;
    int nx, ny, nz;
    long N;
    int bc[3];
    double tau, omega;
    double F[3];
    int comp;           /* 1: weakly compressible equilibrium of Eq. (feq) */
    unsigned char* geo; /* SetGeometry: 1 = fluid, 0 = solid */
    double* f;          /* post-propagation populations, AoS */
    double* fb;         /* post-collision populations, AoS */
    double* rho;        /* PostProcessing: sum_a f_a */
    double* u;          /* PostProcessing: velocity, AoS [id*3 + d] */
};

static long node_id(const orc_sim* s, int x, int y, int z)
{
    return (long)x + (long)s->nx * ((long)y + (long)s->ny * (long)z);
}

#define ORC_WALL (-1)   /* x + sgn e_a is solid, or outside on a halfway-wall axis */
#define ORC_BEYOND (-2) /* x + sgn e_a lies beyond a wall of the modified nodal scheme */

/*
 * The node x + sgn*e_a seen from (x, y, z): wrapped on periodic axes,
 * ORC_BEYOND if it lies outside the box along the axis with nodal walls,
 * ORC_WALL if it lies outside along another wall axis or is solid.
 */
static long neighbour(const orc_sim* s, int x, int y, int z, int a, int sgn)
{
    int c[3] = {x + sgn * s->L.e[a][0], y + sgn * s->L.e[a][1], z + sgn * s->L.e[a][2]};
    int n[3] = {s->nx, s->ny, s->nz};
    for (int d = 0; d < 3; ++d)
        if (s->bc[d] == ORC_WALLS_NODAL && (c[d] < 0 || c[d] >= n[d])) return ORC_BEYOND;
    for (int d = 0; d < 3; ++d) {
        if (c[d] >= 0 && c[d] < n[d]) continue;
        if (s->bc[d] == ORC_PERIODIC)
            c[d] = (c[d] % n[d] + n[d]) % n[d];
        else
            return ORC_WALL;
    }
    long id = node_id(s, c[0], c[1], c[2]);
    return s->geo[id] ? id : ORC_WALL;
}

/*
 * Where the propagation takes f_a(x) from: the slot (node, dir) of the
 * post-collision array.
 *  - Eq. (propagation): fb_a(x - e_a) when x - e_a is a fluid node.
 *  - Eq. (bb), halfway (link-wise) reading: fb_abar(x) when x - e_a is solid
 *    or outside on a halfway-wall axis.
 *  - Eq. (bb), modified nodal reading (Sec. 2.2): on a wall node of the
 *    nodal scheme the population whose source lies beyond the wall is
 *    unknown after the propagation and is replaced by the one that arrived
 *    in the opposite direction, f_a(x) = f_abar(x), i.e. the source of abar.
 *    abar itself points beyond the wall, so its source is inside the box
 *    along that axis and the rule does not recurse further.
 */
static void pull_source(const orc_sim* s, int x, int y, int z, int a, long* node, int* dir)
{
    long id = node_id(s, x, y, z);
    long src = neighbour(s, x, y, z, a, -1);
    if (src == ORC_BEYOND) {
        a = opposite(&s->L, a);
        src = neighbour(s, x, y, z, a, -1);
    }
    if (src >= 0) {
        *node = src;
        *dir = a;
    } else {
        *node = id;
        *dir = opposite(&s->L, a);
    }
}

/* Eq. (bb) on the wall nodes of the nodal scheme: the unknown populations of
 * a post-propagation state are copies of the opposite ones. */
static void nodal_fill_r(const orc_sim* s, double* f)
{
    const int Q = s->L.Q;
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                long id = node_id(s, x, y, z);
                if (!s->geo[id]) continue;
                for (int a = 0; a < Q; ++a)
                    if (neighbour(s, x, y, z, a, -1) == ORC_BEYOND)
                        f[id * Q + a] = f[id * Q + opposite(&s->L, a)];
            }
}

static void nodal_fill_c(const orc_sim* s, double complex* f)
{
    const int Q = s->L.Q;
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                long id = node_id(s, x, y, z);
                if (!s->geo[id]) continue;
                for (int a = 0; a < Q; ++a)
                    if (neighbour(s, x, y, z, a, -1) == ORC_BEYOND)
                        f[id * Q + a] = f[id * Q + opposite(&s->L, a)];
            }
}

static int validate(int lattice, int nx, int ny, int nz, double tau, const double F[3],
                    const int bc[3])
{
    orc_lattice L;
    if (make_lattice(lattice, &L)) return ORC_EINVAL;
    int n[3] = {nx, ny, nz};
    int nodal = 0;
    for (int d = 0; d < 3; ++d) {
        if (n[d] < 1) return ORC_EINVAL;
        if (bc[d] != ORC_PERIODIC && bc[d] != ORC_SOLID_ENDS && bc[d] != ORC_WALLS_OUTSIDE &&
            bc[d] != ORC_WALLS_NODAL)
            return ORC_EINVAL;
        if ((bc[d] == ORC_SOLID_ENDS || bc[d] == ORC_WALLS_NODAL) && n[d] < 3) return ORC_EINVAL;
        nodal += bc[d] == ORC_WALLS_NODAL;
        if (!isfinite(F[d])) return ORC_EINVAL;
    }
    /* One axis at most: on an edge shared by two nodal walls the unknown
     * populations would be defined in terms of each other. */
    if (nodal > 1) return ORC_EINVAL;
    if (lattice == ORC_D2Q9 && (nz != 1 || bc[2] != ORC_PERIODIC || F[2] != 0.0))
        return ORC_EINVAL;
    if (!(tau > 0.5)) return ORC_EINVAL; /* +inf allowed: omega = 0 */
    return 0;
}

int orc_create(int lattice, int nx, int ny, int nz, double tau, const double F[3],
               const int bc[3], orc_sim** out)
{
    *out = NULL;
    int st = validate(lattice, nx, ny, nz, tau, F, bc);
    if (st) return st;
    orc_sim* s = calloc(1, sizeof(orc_sim));
    if (!s) return ORC_ENOMEM;
    make_lattice(lattice, &s->L);
    s->nx = nx;
    s->ny = ny;
    s->nz = nz;
    s->N = (long)nx * ny * nz;
    for (int d = 0; d < 3; ++d) {
        s->bc[d] = bc[d];
        s->F[d] = F[d];
    }
    s->tau = tau;
    s->omega = 1.0 / tau; /* Eq. (collision): 1/(tau_paper/dt + 1/2) with tau = tau_paper + 1/2 */
    const int Q = s->L.Q;
    s->geo = malloc((size_t)s->N);
    s->f = calloc((size_t)s->N * Q, sizeof(double));
    s->fb = calloc((size_t)s->N * Q, sizeof(double));
    s->rho = calloc((size_t)s->N, sizeof(double));
    s->u = calloc((size_t)s->N * 3, sizeof(double));
    if (!s->geo || !s->f || !s->fb || !s->rho || !s->u) {
        orc_destroy(s);
        return ORC_ENOMEM;
    }
    /* SetGeometry: a node is solid when it sits on the first or last plane of
     * an axis whose ends are solid walls. */
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int c[3] = {x, y, z}, n[3] = {nx, ny, nz};
                unsigned char fluid = 1;
                for (int d = 0; d < 3; ++d)
                    if (bc[d] == ORC_SOLID_ENDS && (c[d] == 0 || c[d] == n[d] - 1)) fluid = 0;
                s->geo[node_id(s, x, y, z)] = fluid;
            }
    *out = s;
    return 0;
}

void orc_destroy(orc_sim* s)
{
    if (!s) return;
    free(s->geo);
    free(s->f);
    free(s->fb);
    free(s->rho);
    free(s->u);
    free(s);
}

/* PostProcessing (Sec. 3.1, Table 6): rho and u of every fluid node. */
static void post_processing(orc_sim* s)
{
    const int Q = s->L.Q;
#pragma omp parallel for schedule(static)
    for (long id = 0; id < s->N; ++id) {
        if (!s->geo[id]) {
            s->rho[id] = 0.0;
            s->u[id * 3 + 0] = s->u[id * 3 + 1] = s->u[id * 3 + 2] = 0.0;
            continue;
        }
        node_moments_r(&s->L, s->F, s->f + id * Q, s->comp, s->rho + id, s->u + id * 3);
    }
}

/* Collision (Sec. 3.6 listing, Eq. (collision)): f -> fb on fluid nodes,
 * using rho and u from the preceding PostProcessing. */
static void collision(orc_sim* s)
{
    const int Q = s->L.Q;
#pragma omp parallel for schedule(static)
    for (long id = 0; id < s->N; ++id) {
        if (!s->geo[id]) continue;
        node_relax_r(&s->L, s->omega, s->F, s->rho[id], s->u + id * 3, s->comp, s->f + id * Q,
                     s->fb + id * Q);
    }
}

/*
 * BoundaryCondition + Propagation (Eq. (bb), Eq. (propagation)): each fluid
 * node pulls f_a(x) from the slot that pull_source names.
 */
static void propagation(orc_sim* s)
{
    const int Q = s->L.Q;
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                long id = node_id(s, x, y, z);
                if (!s->geo[id]) continue;
                for (int a = 0; a < Q; ++a) {
                    long node;
                    int dir;
                    pull_source(s, x, y, z, a, &node, &dir);
                    s->f[id * Q + a] = s->fb[node * Q + dir];
                }
            }
}

int orc_init_equilibrium(orc_sim* s, const double* rho, const double* u, const double* noise)
{
    const int Q = s->L.Q;
    const long N = s->N;
    /* InitPDF: f = feq(rho, u) from the given fields (Sec. 2.2), plus an
     * optional perturbation array that is input data. */
    for (long id = 0; id < N; ++id) {
        if (!s->geo[id]) {
            for (int a = 0; a < Q; ++a) s->f[id * Q + a] = 0.0;
            continue;
        }
        double uu[3] = {u[id], u[N + id], u[2 * N + id]};
        double feq[ORC_QMAX];
        node_equilibrium_r(&s->L, rho[id], uu, s->comp, feq);
        for (int a = 0; a < Q; ++a)
            s->f[id * Q + a] = noise ? feq[a] + noise[(long)a * N + id] : feq[a];
    }
    nodal_fill_r(s, s->f);
    post_processing(s);
    return 0;
}

int orc_set_populations(orc_sim* s, const double* f)
{
    const int Q = s->L.Q;
    for (long id = 0; id < s->N; ++id)
        for (int a = 0; a < Q; ++a)
            s->f[id * Q + a] = s->geo[id] ? f[(long)a * s->N + id] : 0.0;
    /* f^n is a post-propagation state: on nodal wall nodes its unknown
     * populations are the opposite ones (Eq. (bb)); given values are ignored. */
    nodal_fill_r(s, s->f);
    post_processing(s);
    return 0;
}

int orc_get_populations(const orc_sim* s, double* f)
{
    const int Q = s->L.Q;
    for (long id = 0; id < s->N; ++id)
        for (int a = 0; a < Q; ++a) f[(long)a * s->N + id] = s->f[id * Q + a];
    return 0;
}

int orc_step(orc_sim* s, int n)
{
    if (n < 0) return ORC_EINVAL;
    for (int it = 0; it < n; ++it) {
        collision(s);
        propagation(s);
        post_processing(s);
    }
    return 0;
}

int orc_moments(const orc_sim* s, double* rho, double* u)
{
    for (long id = 0; id < s->N; ++id) {
        if (rho) rho[id] = s->rho[id];
        if (u)
            for (int d = 0; d < 3; ++d) u[(long)d * s->N + id] = s->u[id * 3 + d];
    }
    return 0;
}

int orc_geometry(const orc_sim* s, unsigned char* geo)
{
    memcpy(geo, s->geo, (size_t)s->N);
    return 0;
}

/*
 * SetGeometry with a user solid mask (Sec. 3.3: geo is 1 on fluid and 0 on
 * solid nodes): a node is fluid when it is not on a solid end plane and
 * solid[id] == 0.  Call before initialising the populations.
 */
int orc_set_solid(orc_sim* s, const unsigned char* solid)
{
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                int c[3] = {x, y, z}, n[3] = {s->nx, s->ny, s->nz};
                unsigned char fluid = 1;
                for (int d = 0; d < 3; ++d)
                    if (s->bc[d] == ORC_SOLID_ENDS && (c[d] == 0 || c[d] == n[d] - 1)) fluid = 0;
                long id = node_id(s, x, y, z);
                if (solid[id]) fluid = 0;
                s->geo[id] = fluid;
            }
    return 0;
}

/*
 * Momentum-exchange force on the walls during the last propagation
 * (Sec. 4, drag evaluation): for every fluid node x and outgoing direction
 * a whose neighbour x + e_a is a wall, the population f*_a(x) that left and
 * the population f_abar(x) that came back carry momentum to the wall:
 *   F = sum_x sum_a [f*_a(x, t) + f_abar(x, t + dt)] e_a.
 * Reading: with the link-wise bounce-back the returning population is the
 * one at x after the propagation (the paper writes it at the wall-side
 * node of the nodal scheme).  Links that cross a wall of the nodal scheme
 * are not part of the sum.
 */
int orc_wall_force(const orc_sim* s, double F[3])
{
    const int Q = s->L.Q;
    kahan acc[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                long id = node_id(s, x, y, z);
                if (!s->geo[id]) continue;
                for (int a = 0; a < Q; ++a) {
                    if (neighbour(s, x, y, z, a, +1) != ORC_WALL) continue;
                    double m = s->fb[id * Q + a] + s->f[id * Q + opposite(&s->L, a)];
                    for (int d = 0; d < 3; ++d) kahan_add(&acc[d], m * (double)s->L.e[a][d]);
                }
            }
    for (int d = 0; d < 3; ++d) F[d] = acc[d].sum + acc[d].comp;
    return 0;
}

/*
 * Monitor analogue (Sec. 3.6): total mass sum rho, kinetic energy
 * sum (rho_m/2) |u|^2 (rho_m = rho0 in the incompressible model, rho in the
 * compressible one) and max |u| over every fluid node, plus the number of
 * non-finite populations.
 */
int orc_reduce(const orc_sim* s, double* mass, double* ke, double* umax, long* nonfinite)
{
    kahan m = {0, 0}, k = {0, 0};
    double um = 0.0;
    long bad = 0;
    const int Q = s->L.Q;
    for (long id = 0; id < s->N; ++id) {
        if (!s->geo[id]) continue;
        for (int a = 0; a < Q; ++a)
            if (!isfinite(s->f[id * Q + a])) ++bad;
        const double* u = s->u + id * 3;
        double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        kahan_add(&m, s->rho[id]);
        kahan_add(&k, 0.5 * (s->comp ? s->rho[id] : ORC_RHO0) * uu);
        if (sqrt(uu) > um) um = sqrt(uu);
    }
    if (mass) *mass = m.sum + m.comp;
    if (ke) *ke = k.sum + k.comp;
    if (umax) *umax = um;
    if (nonfinite) *nonfinite = bad;
    return 0;
}

/* Selects the weakly compressible equilibrium of Eq. (feq) (comp != 0) or
 * the incompressible one of Eq. (incompressible_feq) (comp == 0, the
 * default); call before initialising the populations. */
int orc_set_compressible(orc_sim* s, int comp)
{
    s->comp = comp ? 1 : 0;
    return 0;
}

/* Threads the oracle's parallel loops use (reported with its timings). */
int orc_num_threads(void) { return omp_get_max_threads(); }

/* Sets the thread count of the parallel loops (n >= 1). */
int orc_set_num_threads(int n)
{
    if (n < 1) return ORC_EINVAL;
    omp_set_num_threads(n);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Node-level entry points for the pins.                                     */

int orc_lattice_tables(int lattice, int* Q, int* D, int* e, double* t)
{
    orc_lattice L;
    if (make_lattice(lattice, &L)) return ORC_EINVAL;
    *Q = L.Q;
    *D = L.D;
    for (int a = 0; a < L.Q; ++a) {
        if (e)
            for (int d = 0; d < 3; ++d) e[a * 3 + d] = L.e[a][d];
        if (t) t[a] = L.t[a];
    }
    return 0;
}

int orc_equilibrium_node(int lattice, double rho, const double u[3], int comp, double* feq)
{
    orc_lattice L;
    if (make_lattice(lattice, &L)) return ORC_EINVAL;
    node_equilibrium_r(&L, rho, u, comp, feq);
    return 0;
}

int orc_collide_node(int lattice, double tau, const double F[3], int comp, const double* f,
                     double* fb)
{
    orc_lattice L;
    if (make_lattice(lattice, &L)) return ORC_EINVAL;
    node_collide_r(&L, 1.0 / tau, F, comp, f, fb);
    return 0;
}

int orc_collide_node_cs(int lattice, const double tau[2], const double F[6], const double* f,
                        double* fb)
{
    orc_lattice L;
    if (make_lattice(lattice, &L)) return ORC_EINVAL;
    double complex Fc[3], fc[ORC_QMAX], out[ORC_QMAX];
    for (int d = 0; d < 3; ++d) Fc[d] = CMPLX(F[2 * d], F[2 * d + 1]);
    for (int a = 0; a < L.Q; ++a) fc[a] = CMPLX(f[2 * a], f[2 * a + 1]);
    node_collide_c(&L, 1.0 / CMPLX(tau[0], tau[1]), Fc, 0, fc, out);
    for (int a = 0; a < L.Q; ++a) {
        fb[2 * a] = creal(out[a]);
        fb[2 * a + 1] = cimag(out[a]);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Derivatives: complex-step tangent of the whole run, and the discrete      */
/* adjoint built from complex-step Jacobians of the collision.               */

/* Creates the simulation the derivative entry points run on. */
static int make_sim(int lattice, int nx, int ny, int nz, double tau, const double F[3],
                    const int bc[3], const unsigned char* solid, int comp, orc_sim** out)
{
    int st = orc_create(lattice, nx, ny, nz, tau, F, bc, out);
    if (st) return st;
    if (solid) orc_set_solid(*out, solid);
    orc_set_compressible(*out, comp);
    return 0;
}

/*
 * Tangent by the complex step: runs the forward model in complex arithmetic
 * with
 *   tau + i h dtau,  F + i h dF,  u0 + i h du0
 * and evaluates J = 1/2 sum_x sum_d (u_d^N(x) - u_tgt,d(x))^2 over the fluid
 * nodes.  Re J is the objective, Im J / h its derivative along (du0, dtau, dF)
 * to rounding (the step is rational in f, u0, F and tau).
 */
int orc_cs_objective(int lattice, int nx, int ny, int nz, double tau, double dtau,
                     const double F[3], const double dF[3], const int bc[3],
                     const unsigned char* solid, int comp, const double* rho0, const double* u0,
                     const double* du0, const double* noise, int nsteps, double h,
                     const double* u_tgt, double* J, double* dJ)
{
    orc_sim* s;
    int st = make_sim(lattice, nx, ny, nz, tau, F, bc, solid, comp, &s);
    if (st) return st;
    const int Q = s->L.Q;
    const long N = s->N;
    double complex* f = malloc(sizeof(double complex) * (size_t)N * Q);
    double complex* fb = malloc(sizeof(double complex) * (size_t)N * Q);
    if (!f || !fb) {
        free(f);
        free(fb);
        orc_destroy(s);
        return ORC_ENOMEM;
    }
    double complex omega = 1.0 / CMPLX(tau, h * dtau);
    double complex Fc[3];
    for (int d = 0; d < 3; ++d) Fc[d] = CMPLX(F[d], h * dF[d]);

    for (long id = 0; id < N; ++id) {
        if (!s->geo[id]) {
            for (int a = 0; a < Q; ++a) f[id * Q + a] = 0.0;
            continue;
        }
        double complex uu[3], feq[ORC_QMAX];
        for (int d = 0; d < 3; ++d) uu[d] = CMPLX(u0[d * N + id], h * du0[d * N + id]);
        node_equilibrium_c(&s->L, rho0[id], uu, s->comp, feq);
        for (int a = 0; a < Q; ++a)
            f[id * Q + a] = noise ? feq[a] + noise[(long)a * N + id] : feq[a];
    }
    nodal_fill_c(s, f);
    for (int it = 0; it < nsteps; ++it) {
#pragma omp parallel for schedule(static)
        for (long id = 0; id < N; ++id)
            if (s->geo[id]) node_collide_c(&s->L, omega, Fc, s->comp, f + id * Q, fb + id * Q);
#pragma omp parallel for collapse(2) schedule(static)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    long id = node_id(s, x, y, z);
                    if (!s->geo[id]) continue;
                    for (int a = 0; a < Q; ++a) {
                        long node;
                        int dir;
                        pull_source(s, x, y, z, a, &node, &dir);
                        f[id * Q + a] = fb[node * Q + dir];
                    }
                }
    }
    double complex acc = 0.0;
    for (long id = 0; id < N; ++id) {
        if (!s->geo[id]) continue;
        double complex r, uN[3];
        node_moments_c(&s->L, Fc, f + id * Q, s->comp, &r, uN);
        for (int d = 0; d < s->L.D; ++d) {
            double complex diff = uN[d] - u_tgt[d * N + id];
            acc = acc + 0.5 * diff * diff;
        }
    }
    *J = creal(acc);
    *dJ = cimag(acc) / h;
    free(f);
    free(fb);
    orc_destroy(s);
    return 0;
}

#define ORC_CS_H 1e-30

/*
 * Discrete adjoint of n steps.  Forward: f^0 = B(feq(rho_init, u0) + noise),
 * f^{k+1} = P(C(f^k; tau, F)), u^n = (sum_a e_a f^n_a + F/2)/rho_m, where C
 * is the node collision, P the propagation (a linear map that reads one
 * post-collision slot per population, see pull_source) and B the nodal
 * replacement of Eq. (bb) (the identity without nodal walls).  Given
 * ubar = dJ/du^n, returns dJ/du0, dJ/dtau and dJ/dF by running the
 * transposed steps backwards:
 *   lambda^n   = (du^n/df^n)^T ubar,         Fbar  = (du^n/dF)^T ubar
 *   lambda*    = P^T lambda^{k+1}            (scatter-add along the pulls)
 *   lambda^k   = (dC/df)^T lambda*,  taubar += (dC/dtau)^T lambda*,
 *                                    Fbar   += (dC/dF)^T lambda*
 *   u0bar      = (dfeq/du0)^T B^T lambda^0
 * with every Jacobian column taken by a complex step of h = 1e-30.
 */
int orc_adjoint(int lattice, int nx, int ny, int nz, double tau, const double F[3],
                const int bc[3], const unsigned char* solid, int comp, const double* rho0,
                const double* u0, const double* noise, int nsteps, const double* ubar,
                double* u0bar, double* taubar, double Fbar[3])
{
    if (nsteps < 0) return ORC_EINVAL;
    orc_sim* s;
    int st = make_sim(lattice, nx, ny, nz, tau, F, bc, solid, comp, &s);
    if (st) return st;
    const orc_lattice* L = &s->L;
    const int Q = L->Q;
    const long N = s->N;
    const double h = ORC_CS_H;
    const size_t state = (size_t)N * Q;
    double* traj = malloc(sizeof(double) * state * (size_t)(nsteps + 1));
    double* lam = malloc(sizeof(double) * state);
    double* lstar = malloc(sizeof(double) * state);
    if (!traj || !lam || !lstar) {
        free(traj);
        free(lam);
        free(lstar);
        orc_destroy(s);
        return ORC_ENOMEM;
    }
    orc_init_equilibrium(s, rho0, u0, noise);
    memcpy(traj, s->f, sizeof(double) * state);
    for (int k = 0; k < nsteps; ++k) {
        orc_step(s, 1);
        memcpy(traj + state * (size_t)(k + 1), s->f, sizeof(double) * state);
    }

    double tb = 0.0, Fb[3] = {0.0, 0.0, 0.0};
    const double complex om = 1.0 / tau;
    const double complex Fc[3] = {F[0], F[1], F[2]};
    /* Output map: u^n of every fluid node as a function of f^n and F. */
    {
        const double* fn = traj + state * (size_t)nsteps;
        for (long id = 0; id < N; ++id) {
            for (int a = 0; a < Q; ++a) lam[id * Q + a] = 0.0;
            if (!s->geo[id]) continue;
            double complex fc[ORC_QMAX], r, uN[3];
            for (int b = 0; b < Q; ++b) {
                for (int a = 0; a < Q; ++a) fc[a] = fn[id * Q + a];
                fc[b] = CMPLX(fn[id * Q + b], h);
                node_moments_c(L, Fc, fc, s->comp, &r, uN);
                double acc = 0.0;
                for (int d = 0; d < L->D; ++d) acc = acc + cimag(uN[d]) / h * ubar[d * N + id];
                lam[id * Q + b] = acc;
            }
            for (int a = 0; a < Q; ++a) fc[a] = fn[id * Q + a];
            for (int d = 0; d < L->D; ++d) {
                double complex Fp[3] = {F[0], F[1], F[2]};
                Fp[d] = CMPLX(F[d], h);
                node_moments_c(L, Fp, fc, s->comp, &r, uN);
                for (int e = 0; e < L->D; ++e)
                    Fb[d] = Fb[d] + cimag(uN[e]) / h * ubar[e * N + id];
            }
        }
    }

    for (int k = nsteps - 1; k >= 0; --k) {
        const double* fk = traj + state * (size_t)k;
        /* P^T: every population pulled from slot (node, dir) sends its
         * adjoint back there. */
        for (size_t i = 0; i < state; ++i) lstar[i] = 0.0;
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    long id = node_id(s, x, y, z);
                    if (!s->geo[id]) continue;
                    for (int a = 0; a < Q; ++a) {
                        long node;
                        int dir;
                        pull_source(s, x, y, z, a, &node, &dir);
                        lstar[node * Q + dir] = lstar[node * Q + dir] + lam[id * Q + a];
                    }
                }
        double tb_step = 0.0, Fb_step[3] = {0.0, 0.0, 0.0};
        for (long id = 0; id < N; ++id) {
            if (!s->geo[id]) {
                for (int a = 0; a < Q; ++a) lam[id * Q + a] = 0.0;
                continue;
            }
            const double* ls = lstar + id * Q;
            double complex fc[ORC_QMAX], out[ORC_QMAX];
            /* (dC/df)^T lambda*: column b of dC/df from C(f + i h e_b). */
            for (int b = 0; b < Q; ++b) {
                for (int a = 0; a < Q; ++a) fc[a] = fk[id * Q + a];
                fc[b] = CMPLX(fk[id * Q + b], h);
                node_collide_c(L, om, Fc, s->comp, fc, out);
                double acc = 0.0;
                for (int a = 0; a < Q; ++a) acc = acc + cimag(out[a]) / h * ls[a];
                lam[id * Q + b] = acc;
            }
            for (int a = 0; a < Q; ++a) fc[a] = fk[id * Q + a];
            /* (dC/dtau)^T lambda* */
            node_collide_c(L, 1.0 / CMPLX(tau, h), Fc, s->comp, fc, out);
            for (int a = 0; a < Q; ++a) tb_step = tb_step + cimag(out[a]) / h * ls[a];
            /* (dC/dF)^T lambda* */
            for (int d = 0; d < L->D; ++d) {
                double complex Fp[3] = {F[0], F[1], F[2]};
                Fp[d] = CMPLX(F[d], h);
                node_collide_c(L, om, Fp, s->comp, fc, out);
                for (int a = 0; a < Q; ++a) Fb_step[d] = Fb_step[d] + cimag(out[a]) / h * ls[a];
            }
        }
        tb = tb + tb_step;
        for (int d = 0; d < 3; ++d) Fb[d] = Fb[d] + Fb_step[d];
    }

    /* B^T: an unknown population of a nodal wall node is a copy of the
     * opposite one. */
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long id = node_id(s, x, y, z);
                if (!s->geo[id]) continue;
                for (int a = 0; a < Q; ++a)
                    if (neighbour(s, x, y, z, a, -1) == ORC_BEYOND) {
                        const int abar = opposite(L, a);
                        lam[id * Q + abar] = lam[id * Q + abar] + lam[id * Q + a];
                        lam[id * Q + a] = 0.0;
                    }
            }
    /* Init map: f^0_a = feq_a(rho_init, u0); u0bar = (dfeq/du0)^T lambda^0. */
    for (long id = 0; id < N; ++id) {
        for (int d = 0; d < 3; ++d) u0bar[d * N + id] = 0.0;
        if (!s->geo[id]) continue;
        for (int d = 0; d < L->D; ++d) {
            double complex uu[3] = {u0[id], u0[N + id], u0[2 * N + id]};
            double complex feq[ORC_QMAX];
            uu[d] = CMPLX(u0[d * N + id], h);
            node_equilibrium_c(L, rho0[id], uu, s->comp, feq);
            double acc = 0.0;
            for (int a = 0; a < Q; ++a) acc = acc + cimag(feq[a]) / h * lam[id * Q + a];
            u0bar[d * N + id] = acc;
        }
    }
    *taubar = tb;
    for (int d = 0; d < 3; ++d) Fbar[d] = Fb[d];
    free(traj);
    free(lam);
    free(lstar);
    orc_destroy(s);
    return 0;
}
