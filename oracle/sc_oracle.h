/*
 * sc_oracle.h -- FP64 CPU oracle of the two-component Shan-Chen lattice
 * Boltzmann update (Montella, Yuan, Chareyre, Gens, "A Hybrid multiphase
 * model based on lattice Boltzmann method direct simulations", Sec. 2.1,
 * Eq. 1-5) and of the per-throat drainage ramp (Sec. 2.2.2).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this library; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header, table or helper with the
 * HIP library: it has its own types, its own lattice tables and its own
 * voxelizer, written from the paper and the readings listed in the design
 * notes.
 *
 * Units are lattice units (dx = dt = 1).  Components: 0 = wetting (w),
 * 1 = non-wetting (nw).  Layout of every per-node array: x fastest, then y,
 * then z; population arrays are [component][direction][z][y][x].
 *
 * All functions return 0 on success and a negative code on error; on error
 * the outputs are left untouched.
 */
#ifndef SC_ORACLE_H
#define SC_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* boundary kinds per axis */
#define ORC_PERIODIC 0
#define ORC_WALLS 1     /* nodes beyond the box are solid                  */
#define ORC_RESERVOIR 2 /* z only: planes z=0 / z=nz-1 are density baths   */

/* node classes */
#define ORC_FLUID 0
#define ORC_SOLID 1
#define ORC_RES_IN 2  /* z = 0 plane, non-wetting bath  */
#define ORC_RES_OUT 3 /* z = nz-1 plane, wetting bath   */

/* ramp-point status */
#define ORC_CONVERGED 0
#define ORC_NOT_CONVERGED 1

typedef struct {
  int nx, ny, nz;
  int bc_x, bc_y, bc_z;
  int n_spheres;
  const double *spheres;   /* [n_spheres][4] = cx, cy, cz, r              */
  int prism;               /* 1: solid outside the z-prism over 3 centres */
  int prism_ids[3];
  double tau[2];           /* relaxation times, Eq. 1                      */
  double G;                /* cohesion strength, Eq. 4-5                   */
  double G_ads[2];         /* adhesion strength per component              */
  double rho_major;        /* majority density of a bulk phase             */
  double rho_minor;        /* minority (dissolved) density of a bulk phase */
  double rho_in_nw;        /* nw density of the inlet bath                 */
  double rho_out_w;        /* w density of the outlet bath                 */
  const double *rho_init;  /* [2][nz][ny][nx] or NULL                      */
  int z_front;             /* used when rho_init is NULL                   */
  int probe[3];            /* pore-body probe node for the invasion test   */
} orc_params;

typedef struct orc_sim orc_sim;

int orc_create(const orc_params *p, orc_sim **out);
void orc_free(orc_sim *s);
int orc_clone(const orc_sim *s, orc_sim **out);
int orc_copy_state(orc_sim *dst, const orc_sim *src);

int orc_step(orc_sim *s, long long nsteps);
int orc_set_rho_in(orc_sim *s, double rho_in_nw);
double orc_rho_in_for_pc(const orc_sim *s, double pc);

long long orc_nodes(const orc_sim *s);
int orc_get_types(const orc_sim *s, unsigned char *types);
int orc_get_f(const orc_sim *s, double *f);
int orc_set_f(orc_sim *s, const double *f);
int orc_get_density(const orc_sim *s, double *rho);
int orc_get_force(const orc_sim *s, double *F);      /* [2][3][N] at current t */
int orc_get_velocity(const orc_sim *s, double *u);   /* [3][N] physical        */
int orc_get_pressure(const orc_sim *s, double *p);   /* [N], Eq. 5             */
int orc_reduce(const orc_sim *s, double *mass2, double *S_w, double *momentum3);
int orc_probe_invaded(const orc_sim *s);

int orc_drain(orc_sim *s, const double *pc, int n_pc, double tol,
              int check_every, long long max_steps, double bisect_rel,
              double *S, long long *steps, int *status, double *pce3,
              int *invaded_at);

/* lattice tables and equilibrium, exported for the lattice-identity tests */
void orc_lattice(int *e /* [19][3] */, double *w /* [19] */, int *opp /* [19] */);
void orc_feq(double rho, const double *u3, double *feq19);

#ifdef __cplusplus
}
#endif
#endif
