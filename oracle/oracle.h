/*
 * C interface of the CPU oracle (lbm_oracle.c).  TEST INFRASTRUCTURE ONLY:
 * used by the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark; never by the product path.
 *
 * Field arguments use the canonical structure-of-arrays order
 * [component][z][y][x] with N = nx*ny*nz nodes: rho is [N], u is [3][N],
 * populations are [Q][N].  All are host double arrays owned by the caller.
 * Every int-returning call returns 0 on success, a negative ORC_* code
 * otherwise.
 */
#ifndef IMEXLBM_ORACLE_H
#define IMEXLBM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_D2Q9 = 0, ORC_D3Q19 = 1, ORC_D3Q27 = 2 };
enum { ORC_PERIODIC = 0, ORC_SOLID_ENDS = 1, ORC_WALLS_OUTSIDE = 2, ORC_WALLS_NODAL = 3 };
enum { ORC_EINVAL = -1, ORC_ENOMEM = -2 };

typedef struct orc_sim orc_sim;

int orc_create(int lattice, int nx, int ny, int nz, double tau, const double F[3],
               const int bc[3], orc_sim** out);
void orc_destroy(orc_sim* s);
int orc_init_equilibrium(orc_sim* s, const double* rho, const double* u, const double* noise);
int orc_set_populations(orc_sim* s, const double* f);
int orc_get_populations(const orc_sim* s, double* f);
int orc_step(orc_sim* s, int n);
int orc_moments(const orc_sim* s, double* rho, double* u);
int orc_geometry(const orc_sim* s, unsigned char* geo);
int orc_set_solid(orc_sim* s, const unsigned char* solid);
int orc_wall_force(const orc_sim* s, double F[3]);
int orc_reduce(const orc_sim* s, double* mass, double* ke, double* umax, long* nonfinite);

int orc_num_threads(void);
int orc_set_num_threads(int n);

int orc_lattice_tables(int lattice, int* Q, int* D, int* e, double* t);
int orc_set_compressible(orc_sim* s, int comp);
int orc_equilibrium_node(int lattice, double rho, const double u[3], int comp, double* feq);
int orc_collide_node(int lattice, double tau, const double F[3], int comp, const double* f,
                     double* fb);
/* Complex arguments interleaved (re, im); incompressible model. */
int orc_collide_node_cs(int lattice, const double tau[2], const double F[6], const double* f,
                        double* fb);

/* The derivative entry points take the model flag of orc_set_compressible
 * and an optional solid mask [N] (NULL: none) as orc_set_solid does. */
int orc_cs_objective(int lattice, int nx, int ny, int nz, double tau, double dtau,
                     const double F[3], const double dF[3], const int bc[3],
                     const unsigned char* solid, int comp, const double* rho0, const double* u0,
                     const double* du0, const double* noise, int nsteps, double h,
                     const double* u_tgt, double* J, double* dJ);
int orc_adjoint(int lattice, int nx, int ny, int nz, double tau, const double F[3],
                const int bc[3], const unsigned char* solid, int comp, const double* rho0,
                const double* u0, const double* noise, int nsteps, const double* ubar,
                double* u0bar, double* taubar, double Fbar[3]);

#ifdef __cplusplus
}
#endif
#endif
