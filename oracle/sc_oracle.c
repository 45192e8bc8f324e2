/*
 * sc_oracle.c -- plain FP64 CPU oracle of the two-component Shan-Chen LBM.
 *
 * TEST INFRASTRUCTURE ONLY (see sc_oracle.h).  Slow and direct on purpose:
 * every step below is one loop over the nodes, in the order of Eq. 1 of the
 * paper (collide, then stream), with explicit neighbour tables.  OpenMP only
 * splits node loops whose iterations are independent; every reduction is a
 * serial sum in node order, so results do not depend on the thread count.
 *
 * Readings of the paper taken here (each is listed in the design notes):
 *  - D3Q19 with weights 1/3, 1/18, 1/36 and c_s^2 = 1/3 (Sec. 2.1: D3Q19 is
 *    named, its weights and c_s are not printed).
 *  - Eq. 4 is read as F_s(x) = -G rho_s(x) sum_k w_k rho_sbar(x+e_k) e_k:
 *    potential Psi = rho, cross-component coupling only, D3Q19 weights.  This
 *    is the only reading whose continuum limit gives the pressure of Eq. 5.
 *  - Solid nodes carry zero density in that sum; wetting comes from a
 *    separate adhesion force -G_ads,s rho_s(x) sum_k w_k s(x+e_k) e_k.
 *  - The force enters through the velocity shift of the cited Shan-Chen
 *    model: u' = sum_s (j_s/tau_s) / sum_s (rho_s/tau_s) and
 *    u_eq,s = u' + tau_s F_s / rho_s.
 *  - Second-order polynomial equilibrium, half-way (link-wise) bounce-back,
 *    equilibrium baths on the inlet/outlet planes (Sec. 2.2.2: the density of
 *    the nodes in the inlet and outlet sections is adjusted).
 */
#include "sc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---- D3Q19 velocity set (standard), ordering: rest; +x,-x,+y,-y,+z,-z;
 *      then the twelve edge vectors with each opposite pair adjacent ------- */
static const int E[19][3] = {
    {0, 0, 0},                                                   /* 0 */
    {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},  {0, -1, 0},            /* 1-4 */
    {0, 0, 1},   {0, 0, -1},                                     /* 5-6 */
    {1, 1, 0},   {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},            /* 7-10 */
    {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},            /* 11-14 */
    {0, 1, 1},   {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};           /* 15-18 */

static const double W[19] = {
    1.0 / 3.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

static const double CS2 = 1.0 / 3.0;

static int opp(int k) { return k == 0 ? 0 : ((k & 1) ? k + 1 : k - 1); }

struct orc_sim {
  int nx, ny, nz;
  long long N;
  int bc[3];
  double tau[2], G, G_ads[2];
  double rho_major, rho_minor, rho_in_nw, rho_out_w;
  long long probe; /* node index or -1 */
  unsigned char *type; /* [N] */
  long long *nbr;      /* [19][N]: index of x + e_k, or -1 beyond a wall */
  double *f;           /* [2][19][N] pre-collision populations */
  double *fpost;       /* [2][19][N] post-collision scratch    */
  double *rho;         /* [2][N] */
  double *j;           /* [2][3][N] */
  double *F;           /* [2][3][N] */
};

#define IDX(s, x, y, z) ((long long)(x) + (long long)(s)->nx * ((long long)(y) + (long long)(s)->ny * (long long)(z)))

void orc_lattice(int *e, double *w, int *o) {
  for (int k = 0; k < 19; ++k) {
    for (int a = 0; a < 3; ++a) e[3 * k + a] = E[k][a];
    w[k] = W[k];
    o[k] = opp(k);
  }
}

/* f_eq,k = w_k rho [1 + e.u/c_s^2 + (e.u)^2/(2 c_s^4) - u.u/(2 c_s^2)] */
void orc_feq(double rho, const double *u, double *feq) {
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int k = 0; k < 19; ++k) {
    double eu = E[k][0] * u[0] + E[k][1] * u[1] + E[k][2] * u[2];
    feq[k] = W[k] * rho * (1.0 + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
  }
}

/* ---- geometry: node-centred voxelization (node (i,j,k) at integer
 *      coordinates); predicates in FP64, evaluated term by term ---------- */
static int in_sphere(double x, double y, double z, const double *sp) {
  double dx = x - sp[0];
  double dy = y - sp[1];
  double dz = z - sp[2];
  double d2 = dx * dx;
  d2 = d2 + dy * dy;
  d2 = d2 + dz * dz;
  return d2 <= sp[3] * sp[3];
}

static double edge_fn(const double *P, const double *Q, double x, double y) {
  double a = (Q[0] - P[0]) * (y - P[1]);
  double b = (Q[1] - P[1]) * (x - P[0]);
  return a - b;
}

/* inside (boundary included) the triangle of the three sphere centres,
 * projected on the xy-plane: the cross-section of the throat prism */
static int in_prism(double x, double y, const double *A, const double *B, const double *C) {
  double o = edge_fn(A, B, C[0], C[1]);
  double e1 = edge_fn(A, B, x, y), e2 = edge_fn(B, C, x, y), e3 = edge_fn(C, A, x, y);
  if (o > 0) return e1 >= 0 && e2 >= 0 && e3 >= 0;
  return e1 <= 0 && e2 <= 0 && e3 <= 0;
}

static int finite_pos(double v) { return isfinite(v) && v > 0; }

static int validate(const orc_params *p) {
  if (!p) return -1;
  if (p->nx < 3 || p->ny < 3 || p->nz < 3) return -1;
  if (p->bc_x != ORC_PERIODIC && p->bc_x != ORC_WALLS) return -1;
  if (p->bc_y != ORC_PERIODIC && p->bc_y != ORC_WALLS) return -1;
  if (p->bc_z != ORC_PERIODIC && p->bc_z != ORC_WALLS && p->bc_z != ORC_RESERVOIR) return -1;
  if (!(p->tau[0] > 0.5) || !(p->tau[1] > 0.5) || !isfinite(p->tau[0]) || !isfinite(p->tau[1])) return -1;
  if (!isfinite(p->G) || !isfinite(p->G_ads[0]) || !isfinite(p->G_ads[1])) return -1;
  if (!finite_pos(p->rho_major) || !finite_pos(p->rho_minor)) return -1;
  if (!finite_pos(p->rho_in_nw) || !finite_pos(p->rho_out_w)) return -1;
  if (p->n_spheres < 0 || (p->n_spheres > 0 && !p->spheres)) return -1;
  for (int i = 0; i < p->n_spheres; ++i) {
    for (int a = 0; a < 4; ++a)
      if (!isfinite(p->spheres[4 * i + a])) return -1;
    if (!(p->spheres[4 * i + 3] > 0)) return -1;
  }
  if (p->prism) {
    for (int a = 0; a < 3; ++a)
      if (p->prism_ids[a] < 0 || p->prism_ids[a] >= p->n_spheres) return -1;
  }
  return 0;
}

static void free_arrays(orc_sim *s) {
  if (!s) return;
  free(s->type);
  free(s->nbr);
  free(s->f);
  free(s->fpost);
  free(s->rho);
  free(s->j);
  free(s->F);
}

void orc_free(orc_sim *s) {
  if (!s) return;
  free_arrays(s);
  free(s);
}

static int alloc_arrays(orc_sim *s) {
  long long N = s->N;
  s->type = (unsigned char *)calloc((size_t)N, 1);
  s->nbr = (long long *)malloc(sizeof(long long) * 19 * (size_t)N);
  s->f = (double *)calloc((size_t)(2 * 19 * N), sizeof(double));
  s->fpost = (double *)calloc((size_t)(2 * 19 * N), sizeof(double));
  s->rho = (double *)calloc((size_t)(2 * N), sizeof(double));
  s->j = (double *)calloc((size_t)(6 * N), sizeof(double));
  s->F = (double *)calloc((size_t)(6 * N), sizeof(double));
  if (!s->type || !s->nbr || !s->f || !s->fpost || !s->rho || !s->j || !s->F) return -2;
  return 0;
}

/* reservoir density of component c at a node of class t */
static double res_density(const orc_sim *s, int t, int c) {
  if (t == ORC_RES_IN) return c == 1 ? s->rho_in_nw : s->rho_minor;
  return c == 0 ? s->rho_out_w : s->rho_minor;
}

static void impose_reservoirs(orc_sim *s) {
  long long N = s->N;
  for (long long n = 0; n < N; ++n) {
    int t = s->type[n];
    if (t != ORC_RES_IN && t != ORC_RES_OUT) continue;
    for (int c = 0; c < 2; ++c) {
      double r = res_density(s, t, c);
      for (int k = 0; k < 19; ++k) s->f[((long long)c * 19 + k) * N + n] = W[k] * r;
    }
  }
}

int orc_create(const orc_params *p, orc_sim **out) {
  if (!out || validate(p)) return -1;
  orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
  if (!s) return -2;
  s->nx = p->nx;
  s->ny = p->ny;
  s->nz = p->nz;
  s->N = (long long)p->nx * p->ny * p->nz;
  s->bc[0] = p->bc_x;
  s->bc[1] = p->bc_y;
  s->bc[2] = p->bc_z;
  s->tau[0] = p->tau[0];
  s->tau[1] = p->tau[1];
  s->G = p->G;
  s->G_ads[0] = p->G_ads[0];
  s->G_ads[1] = p->G_ads[1];
  s->rho_major = p->rho_major;
  s->rho_minor = p->rho_minor;
  s->rho_in_nw = p->rho_in_nw;
  s->rho_out_w = p->rho_out_w;
  if (alloc_arrays(s)) {
    orc_free(s);
    return -2;
  }
  long long N = s->N;
  int dims[3] = {s->nx, s->ny, s->nz};

  /* node classes */
  for (int z = 0; z < s->nz; ++z)
    for (int y = 0; y < s->ny; ++y)
      for (int x = 0; x < s->nx; ++x) {
        int solid = 0;
        for (int i = 0; i < p->n_spheres && !solid; ++i)
          solid = in_sphere((double)x, (double)y, (double)z, p->spheres + 4 * i);
        if (!solid && p->prism) {
          const double *A = p->spheres + 4 * p->prism_ids[0];
          const double *B = p->spheres + 4 * p->prism_ids[1];
          const double *C = p->spheres + 4 * p->prism_ids[2];
          solid = !in_prism((double)x, (double)y, A, B, C);
        }
        unsigned char t = ORC_FLUID;
        if (solid) t = ORC_SOLID;
        else if (s->bc[2] == ORC_RESERVOIR && z == 0) t = ORC_RES_IN;
        else if (s->bc[2] == ORC_RESERVOIR && z == s->nz - 1) t = ORC_RES_OUT;
        s->type[IDX(s, x, y, z)] = t;
      }

  /* neighbour table: nbr[k][n] = index of n + e_k (wrapped where periodic),
   * -1 where n + e_k lies beyond a wall or beyond a reservoir plane */
  for (int z = 0; z < s->nz; ++z)
    for (int y = 0; y < s->ny; ++y)
      for (int x = 0; x < s->nx; ++x) {
        long long n = IDX(s, x, y, z);
        for (int k = 0; k < 19; ++k) {
          int c[3] = {x + E[k][0], y + E[k][1], z + E[k][2]};
          int ok = 1;
          for (int a = 0; a < 3; ++a) {
            if (c[a] >= 0 && c[a] < dims[a]) continue;
            if (s->bc[a] == ORC_PERIODIC) c[a] = (c[a] + dims[a]) % dims[a];
            else ok = 0;
          }
          s->nbr[(long long)k * N + n] = ok ? IDX(s, c[0], c[1], c[2]) : -1;
        }
      }

  /* probe */
  s->probe = -1;
  if (p->probe[0] >= 0) {
    if (p->probe[0] >= s->nx || p->probe[1] < 0 || p->probe[1] >= s->ny || p->probe[2] < 0 ||
        p->probe[2] >= s->nz) {
      orc_free(s);
      return -1;
    }
    s->probe = IDX(s, p->probe[0], p->probe[1], p->probe[2]);
    if (s->type[s->probe] != ORC_FLUID) {
      orc_free(s);
      return -1;
    }
  }

  /* initial state: f = f_eq(rho(x,0), u = 0) on fluid nodes */
  for (int z = 0; z < s->nz; ++z)
    for (int y = 0; y < s->ny; ++y)
      for (int x = 0; x < s->nx; ++x) {
        long long n = IDX(s, x, y, z);
        if (s->type[n] != ORC_FLUID) continue;
        for (int c = 0; c < 2; ++c) {
          double r;
          if (p->rho_init) {
            r = p->rho_init[(long long)c * N + n];
          } else {
            int nw_here = z <= p->z_front;
            r = (c == 1) == nw_here ? s->rho_major : s->rho_minor;
          }
          if (!finite_pos(r)) {
            orc_free(s);
            return -1;
          }
          for (int k = 0; k < 19; ++k) s->f[((long long)c * 19 + k) * N + n] = W[k] * r;
        }
      }
  impose_reservoirs(s);
  *out = s;
  return 0;
}

int orc_copy_state(orc_sim *d, const orc_sim *s) {
  if (!d || !s || d->N != s->N) return -1;
  memcpy(d->f, s->f, sizeof(double) * 38 * (size_t)s->N);
  d->rho_in_nw = s->rho_in_nw;
  return 0;
}

int orc_clone(const orc_sim *s, orc_sim **out) {
  if (!s || !out) return -1;
  orc_sim *d = (orc_sim *)calloc(1, sizeof(orc_sim));
  if (!d) return -2;
  *d = *s;
  d->type = NULL;
  d->nbr = NULL;
  d->f = d->fpost = d->rho = d->j = d->F = NULL;
  if (alloc_arrays(d)) {
    orc_free(d);
    return -2;
  }
  memcpy(d->type, s->type, (size_t)s->N);
  memcpy(d->nbr, s->nbr, sizeof(long long) * 19 * (size_t)s->N);
  memcpy(d->f, s->f, sizeof(double) * 38 * (size_t)s->N);
  *out = d;
  return 0;
}

long long orc_nodes(const orc_sim *s) { return s ? s->N : -1; }

/* ---- moments (Eq. 2-3), forces (Eq. 4 + adhesion) at the current state -- */

/* density seen by the interaction sums: zero on solid nodes and beyond walls,
 * the imposed bath value on reservoir nodes */
static double rho_seen(const orc_sim *s, long long m, int c) {
  if (m < 0) return 0.0;
  int t = s->type[m];
  if (t == ORC_SOLID) return 0.0;
  if (t == ORC_FLUID) return s->rho[(long long)c * s->N + m];
  return res_density(s, t, c);
}

static double solid_seen(const orc_sim *s, long long m) {
  if (m < 0) return 1.0;
  return s->type[m] == ORC_SOLID ? 1.0 : 0.0;
}

static void compute_moments(orc_sim *s) {
  long long N = s->N;
#pragma omp parallel for schedule(static)
  for (long long n = 0; n < N; ++n) {
    for (int c = 0; c < 2; ++c) {
      double r = 0, jx = 0, jy = 0, jz = 0;
      if (s->type[n] == ORC_FLUID) {
        for (int k = 0; k < 19; ++k) {
          double fk = s->f[((long long)c * 19 + k) * N + n];
          r += fk;
          jx += fk * E[k][0];
          jy += fk * E[k][1];
          jz += fk * E[k][2];
        }
      } else if (s->type[n] != ORC_SOLID) {
        r = res_density(s, s->type[n], c);
      }
      s->rho[(long long)c * N + n] = r;
      s->j[((long long)c * 3 + 0) * N + n] = jx;
      s->j[((long long)c * 3 + 1) * N + n] = jy;
      s->j[((long long)c * 3 + 2) * N + n] = jz;
    }
  }
}

static void compute_forces(orc_sim *s) {
  long long N = s->N;
#pragma omp parallel for schedule(static)
  for (long long n = 0; n < N; ++n) {
    double Fv[2][3] = {{0, 0, 0}, {0, 0, 0}};
    if (s->type[n] == ORC_FLUID) {
      double Sg[2][3] = {{0, 0, 0}, {0, 0, 0}}, A[3] = {0, 0, 0};
      for (int k = 1; k < 19; ++k) {
        long long m = s->nbr[(long long)k * N + n];
        double sol = solid_seen(s, m);
        for (int c = 0; c < 2; ++c) {
          double r = rho_seen(s, m, c);
          for (int a = 0; a < 3; ++a) Sg[c][a] += W[k] * r * E[k][a];
        }
        for (int a = 0; a < 3; ++a) A[a] += W[k] * sol * E[k][a];
      }
      for (int c = 0; c < 2; ++c) {
        double rc = s->rho[(long long)c * N + n];
        for (int a = 0; a < 3; ++a)
          Fv[c][a] = -s->G * rc * Sg[1 - c][a] - s->G_ads[c] * rc * A[a];
      }
    }
    for (int c = 0; c < 2; ++c)
      for (int a = 0; a < 3; ++a) s->F[((long long)c * 3 + a) * N + n] = Fv[c][a];
  }
}

/* ---- one time step: collide (Eq. 1 right-hand side), then stream -------- */
static void collide(orc_sim *s) {
  long long N = s->N;
#pragma omp parallel for schedule(static)
  for (long long n = 0; n < N; ++n) {
    int t = s->type[n];
    if (t == ORC_SOLID) continue;
    if (t != ORC_FLUID) {
      for (int c = 0; c < 2; ++c) {
        double r = res_density(s, t, c);
        for (int k = 0; k < 19; ++k) s->fpost[((long long)c * 19 + k) * N + n] = W[k] * r;
      }
      continue;
    }
    double num[3] = {0, 0, 0}, den = 0;
    for (int c = 0; c < 2; ++c) {
      for (int a = 0; a < 3; ++a) num[a] += s->j[((long long)c * 3 + a) * N + n] / s->tau[c];
      den += s->rho[(long long)c * N + n] / s->tau[c];
    }
    double up[3] = {num[0] / den, num[1] / den, num[2] / den};
    for (int c = 0; c < 2; ++c) {
      double rc = s->rho[(long long)c * N + n];
      double ueq[3], feq[19];
      for (int a = 0; a < 3; ++a) ueq[a] = up[a] + s->tau[c] * s->F[((long long)c * 3 + a) * N + n] / rc;
      orc_feq(rc, ueq, feq);
      for (int k = 0; k < 19; ++k) {
        long long q = ((long long)c * 19 + k) * N + n;
        s->fpost[q] = s->f[q] - (s->f[q] - feq[k]) / s->tau[c];
      }
    }
  }
}

static void stream(orc_sim *s) {
  long long N = s->N;
#pragma omp parallel for schedule(static)
  for (long long n = 0; n < N; ++n) {
    if (s->type[n] != ORC_FLUID) continue;
    for (int k = 0; k < 19; ++k) {
      long long src = s->nbr[(long long)opp(k) * N + n]; /* n - e_k */
      int bounce = src < 0 || s->type[src] == ORC_SOLID;
      for (int c = 0; c < 2; ++c) {
        double v = bounce ? s->fpost[((long long)c * 19 + opp(k)) * N + n]
                          : s->fpost[((long long)c * 19 + k) * N + src];
        s->f[((long long)c * 19 + k) * N + n] = v;
      }
    }
  }
  impose_reservoirs(s);
}

int orc_step(orc_sim *s, long long nsteps) {
  if (!s || nsteps < 0) return -1;
  for (long long t = 0; t < nsteps; ++t) {
    compute_moments(s);
    compute_forces(s);
    collide(s);
    stream(s);
  }
  return 0;
}

/* ---- observables ------------------------------------------------------ */
int orc_get_types(const orc_sim *s, unsigned char *types) {
  if (!s || !types) return -1;
  memcpy(types, s->type, (size_t)s->N);
  return 0;
}

int orc_get_f(const orc_sim *s, double *f) {
  if (!s || !f) return -1;
  memcpy(f, s->f, sizeof(double) * 38 * (size_t)s->N);
  return 0;
}

int orc_set_f(orc_sim *s, const double *f) {
  if (!s || !f) return -1;
  for (long long q = 0; q < 38 * s->N; ++q)
    if (!isfinite(f[q])) return -1;
  long long N = s->N;
  for (int c = 0; c < 2; ++c)
    for (int k = 0; k < 19; ++k)
      for (long long n = 0; n < N; ++n) {
        long long q = ((long long)c * 19 + k) * N + n;
        s->f[q] = s->type[n] == ORC_FLUID ? f[q] : 0.0;
      }
  impose_reservoirs(s);
  return 0;
}

int orc_get_density(const orc_sim *s, double *rho) {
  if (!s || !rho) return -1;
  compute_moments((orc_sim *)s);
  memcpy(rho, s->rho, sizeof(double) * 2 * (size_t)s->N);
  return 0;
}

int orc_get_force(const orc_sim *s, double *F) {
  if (!s || !F) return -1;
  compute_moments((orc_sim *)s);
  compute_forces((orc_sim *)s);
  memcpy(F, s->F, sizeof(double) * 6 * (size_t)s->N);
  return 0;
}

/* physical velocity: total momentum plus half the total force, over the total
 * density (the velocity carried by the velocity-shift forcing) */
int orc_get_velocity(const orc_sim *s, double *u) {
  if (!s || !u) return -1;
  orc_sim *m = (orc_sim *)s;
  compute_moments(m);
  compute_forces(m);
  long long N = s->N;
  for (long long n = 0; n < N; ++n) {
    double r = s->rho[n] + s->rho[N + n];
    for (int a = 0; a < 3; ++a) {
      double v = 0;
      if (s->type[n] == ORC_FLUID) {
        double jt = s->j[(0 * 3 + a) * N + n] + s->j[(1 * 3 + a) * N + n];
        double Ft = s->F[(0 * 3 + a) * N + n] + s->F[(1 * 3 + a) * N + n];
        v = (jt + 0.5 * Ft) / r;
      }
      u[(long long)a * N + n] = v;
    }
  }
  return 0;
}

/* Eq. 5: p = c_s^2 (rho_w + rho_nw) + c_s^2 G rho_w rho_nw */
int orc_get_pressure(const orc_sim *s, double *p) {
  if (!s || !p) return -1;
  compute_moments((orc_sim *)s);
  long long N = s->N;
  for (long long n = 0; n < N; ++n) {
    double a = s->rho[n], b = s->rho[N + n];
    p[n] = s->type[n] == ORC_SOLID ? 0.0 : CS2 * (a + b) + CS2 * s->G * a * b;
  }
  return 0;
}

/* masses and wetting saturation over fluid nodes; saturation from the local
 * order parameter phi = (rho_w - rho_nw)/(rho_w + rho_nw), mapped linearly so
 * that a pure wetting bulk gives 1 and a pure non-wetting bulk gives 0 */
int orc_reduce(const orc_sim *s, double *mass2, double *S_w, double *mom3) {
  if (!s) return -1;
  compute_moments((orc_sim *)s);
  long long N = s->N;
  double phib = (s->rho_major - s->rho_minor) / (s->rho_major + s->rho_minor);
  double m0 = 0, m1 = 0, acc = 0, P[3] = {0, 0, 0};
  long long cnt = 0;
  for (long long n = 0; n < N; ++n) {
    if (s->type[n] != ORC_FLUID) continue;
    double a = s->rho[n], b = s->rho[N + n];
    m0 += a;
    m1 += b;
    double phi = (a - b) / (a + b);
    acc += (phi + phib) / (2.0 * phib);
    for (int q = 0; q < 3; ++q) P[q] += s->j[(0 * 3 + q) * N + n] + s->j[(1 * 3 + q) * N + n];
    ++cnt;
  }
  if (mass2) {
    mass2[0] = m0;
    mass2[1] = m1;
  }
  if (S_w) *S_w = cnt ? acc / (double)cnt : 0.0;
  if (mom3)
    for (int q = 0; q < 3; ++q) mom3[q] = P[q];
  return 0;
}

/* invaded: non-wetting density exceeds wetting density at the probe node */
int orc_probe_invaded(const orc_sim *s) {
  if (!s || s->probe < 0) return -1;
  compute_moments((orc_sim *)s);
  return s->rho[s->N + s->probe] > s->rho[s->probe] ? 1 : 0;
}

/* ---- drainage ramp (Sec. 2.2.2): the inlet density is raised step by step;
 *      each step runs to steady state; the entry pressure is the threshold
 *      between the last stable and the first invaded step -------------- */
int orc_set_rho_in(orc_sim *s, double r) {
  if (!s || !finite_pos(r)) return -1;
  s->rho_in_nw = r;
  impose_reservoirs(s);
  return 0;
}

/* p_c = p(inlet) - p(outlet) from Eq. 5 with the minority density fixed:
 * c_s^2 (1 + G rho_minor)(rho_in - rho_out) */
double orc_rho_in_for_pc(const orc_sim *s, double pc) {
  return s->rho_out_w + pc / (CS2 * (1.0 + s->G * s->rho_minor));
}

static int run_to_steady(orc_sim *s, double tol, int every, long long cap, double *S_end,
                         long long *used) {
  double S_old, S_new;
  orc_reduce(s, NULL, &S_old, NULL);
  long long n = 0;
  for (;;) {
    orc_step(s, every);
    n += every;
    orc_reduce(s, NULL, &S_new, NULL);
    if (!isfinite(S_new)) {
      *S_end = S_new;
      *used = n;
      return -4;
    }
    if (fabs(S_new - S_old) < tol) {
      *S_end = S_new;
      *used = n;
      return ORC_CONVERGED;
    }
    if (n >= cap) {
      *S_end = S_new;
      *used = n;
      return ORC_NOT_CONVERGED;
    }
    S_old = S_new;
  }
}

int orc_drain(orc_sim *s, const double *pc, int n_pc, double tol, int every, long long cap,
              double bisect_rel, double *S, long long *steps, int *status, double *pce3,
              int *invaded_at) {
  if (!s || !pc || n_pc < 1 || !S || !steps || !status || !pce3 || !invaded_at) return -1;
  if (!(tol > 0) || every < 1 || cap < every || !(bisect_rel > 0) || s->probe < 0) return -1;
  for (int i = 0; i < n_pc; ++i)
    if (!isfinite(pc[i]) || !(pc[i] > 0) || !(orc_rho_in_for_pc(s, pc[i]) > 0)) return -1;
  for (int i = 1; i < n_pc; ++i)
    if (!(pc[i] > pc[i - 1])) return -1;

  orc_sim *stable = NULL; /* last converged, not invaded state */
  if (orc_clone(s, &stable)) return -2;
  double stable_pc = 0.0;
  int inv_at = -1;
  double lo = NAN, hi = NAN;
  for (int i = 0; i < n_pc; ++i) {
    orc_set_rho_in(s, orc_rho_in_for_pc(s, pc[i]));
    int st = run_to_steady(s, tol, every, cap, &S[i], &steps[i]);
    if (st < 0) {
      orc_free(stable);
      return st;
    }
    status[i] = st;
    int inv = orc_probe_invaded(s);
    if (!inv) {
      orc_copy_state(stable, s);
      stable_pc = pc[i];
      continue;
    }
    if (inv_at >= 0) continue;
    inv_at = i;
    /* bisection between the stable state and the first invaded pressure */
    lo = i == 0 ? 0.0 : stable_pc;
    hi = pc[i];
    orc_sim *trial = NULL;
    if (orc_clone(stable, &trial)) {
      orc_free(stable);
      return -2;
    }
    /* at most 40 runs: from a lower bracket of 0 (invaded at pc[0]) halving
       alone need not reach the relative width */
    for (int runs = 0; (hi - lo) / hi > bisect_rel && runs < 40; ++runs) {
      double mid = 0.5 * (lo + hi);
      double Sm;
      long long nm;
      orc_copy_state(trial, stable);
      orc_set_rho_in(trial, orc_rho_in_for_pc(trial, mid));
      int sm = run_to_steady(trial, tol, every, cap, &Sm, &nm);
      if (sm < 0) {
        orc_free(trial);
        orc_free(stable);
        return sm;
      }
      if (orc_probe_invaded(trial)) {
        hi = mid;
      } else {
        lo = mid;
        orc_copy_state(stable, trial);
      }
    }
    orc_free(trial);
  }
  orc_free(stable);
  *invaded_at = inv_at;
  if (inv_at < 0) {
    pce3[0] = pc[n_pc - 1];
    pce3[1] = NAN;
    pce3[2] = INFINITY;
  } else {
    pce3[0] = lo;
    pce3[1] = 0.5 * (lo + hi);
    pce3[2] = hi;
  }
  return 0;
}
