/*
 * lbm_drain -- drainage of one pore-throat subdomain from the command line,
 * through the C interface of lbm_abi.h only (no Python).
 *
 *   lbm_drain PROBLEM [--checkpoint PATH] [--chunk STEPS] [--max-chunks K]
 *
 * PROBLEM is a text file stating the subdomain and its ramp (Sec. 2.1-2.2.2:
 * geometry, densities, relaxation times, interaction strengths, the imposed
 * capillary pressures and the steady-state test), one keyword per line
 * ('#' starts a comment):
 *
 *   size NX NY NZ            bc BX BY BZ (LBM_BC_*)     tau TAU_W TAU_NW
 *   G G                      G_ads GW GNW                rho MAJOR MINOR
 *   baths RHO_IN_NW RHO_OUT_W                            z_front Z
 *   probe X Y Z              prism I0 I1 I2 (optional)
 *   sphere CX CY CZ R (one line per sphere)
 *   pc P0 P1 ... (strictly increasing)
 *   conv TOL CHECK_EVERY MAX_STEPS BISECT_REL
 *
 * The ramp runs with lbm_drain_begin / lbm_drain_advance in chunks of STEPS
 * lattice steps (default 10000).  With --checkpoint, the handle is saved
 * after every chunk (to PATH.tmp, then renamed over PATH), and a run that
 * finds PATH loads it and continues the ramp where the saved run stopped:
 * the results are those of an uninterrupted drain, bit for bit.
 * --max-chunks stops after K chunks (exit status 3, the checkpoint written).
 *
 * Output (stdout): the drainage result as "key value..." lines, numbers with
 * 17 significant digits.  Exit status: 0 done, 1 usage or problem-file
 * error, 2 library error (message from lbm_last_error), 3 stopped early.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbm_abi.h"

#define MAX_SPHERES 4096
#define MAX_PC 1024

typedef struct {
  lbm_params p;
  lbm_sphere sph[MAX_SPHERES];
  double pc[MAX_PC];
  int n_pc;
  lbm_conv conv;
} problem;

static int read_doubles(FILE *f, double *v, int n) {
  for (int i = 0; i < n; ++i)
    if (fscanf(f, "%lf", &v[i]) != 1) return 0;
  return 1;
}

static int read_ints(FILE *f, int *v, int n) {
  for (int i = 0; i < n; ++i)
    if (fscanf(f, "%d", &v[i]) != 1) return 0;
  return 1;
}

static int read_problem(const char *path, problem *q) {
  FILE *f = fopen(path, "r");
  if (!f) {
    fprintf(stderr, "lbm_drain: cannot open %s\n", path);
    return 0;
  }
  memset(q, 0, sizeof *q);
  q->p.probe[0] = q->p.probe[1] = q->p.probe[2] = -1;
  char key[32];
  int ok = 1, have_size = 0, have_conv = 0;
  while (ok && fscanf(f, "%31s", key) == 1) {
    if (key[0] == '#') {
      int c;
      while ((c = fgetc(f)) != EOF && c != '\n') {
      }
    } else if (!strcmp(key, "size")) {
      ok = read_ints(f, &q->p.nx, 1) && read_ints(f, &q->p.ny, 1) && read_ints(f, &q->p.nz, 1);
      have_size = ok;
    } else if (!strcmp(key, "bc")) {
      ok = read_ints(f, q->p.bc, 3);
    } else if (!strcmp(key, "tau")) {
      ok = read_doubles(f, q->p.tau, 2);
    } else if (!strcmp(key, "G")) {
      ok = read_doubles(f, &q->p.G, 1);
    } else if (!strcmp(key, "G_ads")) {
      ok = read_doubles(f, q->p.G_ads, 2);
    } else if (!strcmp(key, "rho")) {
      ok = read_doubles(f, &q->p.rho_major, 1) && read_doubles(f, &q->p.rho_minor, 1);
    } else if (!strcmp(key, "baths")) {
      ok = read_doubles(f, &q->p.rho_in_nw, 1) && read_doubles(f, &q->p.rho_out_w, 1);
    } else if (!strcmp(key, "z_front")) {
      ok = read_ints(f, &q->p.z_front, 1);
    } else if (!strcmp(key, "probe")) {
      ok = read_ints(f, q->p.probe, 3);
    } else if (!strcmp(key, "prism")) {
      ok = read_ints(f, q->p.prism_ids, 3);
      q->p.prism = 1;
    } else if (!strcmp(key, "sphere")) {
      ok = q->p.n_spheres < MAX_SPHERES;
      if (ok) {
        lbm_sphere *s = &q->sph[q->p.n_spheres++];
        ok = read_doubles(f, s->c, 3) && read_doubles(f, &s->r, 1);
      }
    } else if (!strcmp(key, "pc")) {
      double v;
      long pos = ftell(f);
      while (q->n_pc < MAX_PC && fscanf(f, "%lf", &v) == 1) {
        q->pc[q->n_pc++] = v;
        pos = ftell(f);
      }
      /* the next keyword stopped the scan: step back to its start */
      ok = q->n_pc > 0 && fseek(f, pos, SEEK_SET) == 0;
    } else if (!strcmp(key, "conv")) {
      ok = read_doubles(f, &q->conv.tol, 1) && read_ints(f, &q->conv.check_every, 1) &&
           fscanf(f, "%lld", &q->conv.max_steps) == 1 && read_doubles(f, &q->conv.bisect_rel, 1);
      have_conv = ok;
    } else {
      fprintf(stderr, "lbm_drain: unknown keyword '%s' in %s\n", key, path);
      ok = 0;
    }
  }
  fclose(f);
  if (!ok || !have_size || !have_conv || q->n_pc < 1) {
    fprintf(stderr, "lbm_drain: %s is incomplete or malformed (size, pc and conv are required)\n",
            path);
    return 0;
  }
  q->p.spheres = q->sph;
  return 1;
}

static int fail(const char *what, int rc) {
  fprintf(stderr, "lbm_drain: %s failed (%d): %s\n", what, rc, lbm_last_error());
  return 2;
}

static int file_exists(const char *path) {
  FILE *f = fopen(path, "rb");
  if (!f) return 0;
  fclose(f);
  return 1;
}

int main(int argc, char **argv) {
  const char *prob_path = NULL, *ckpt = NULL;
  long long chunk = 10000, max_chunks = -1;
  for (int i = 1; i < argc; ++i) {
    if (!strcmp(argv[i], "--checkpoint") && i + 1 < argc) {
      ckpt = argv[++i];
    } else if (!strcmp(argv[i], "--chunk") && i + 1 < argc) {
      chunk = atoll(argv[++i]);
    } else if (!strcmp(argv[i], "--max-chunks") && i + 1 < argc) {
      max_chunks = atoll(argv[++i]);
    } else if (argv[i][0] != '-' && !prob_path) {
      prob_path = argv[i];
    } else {
      prob_path = NULL;
      break;
    }
  }
  if (!prob_path || chunk < 1) {
    fprintf(stderr,
            "usage: lbm_drain PROBLEM [--checkpoint PATH] [--chunk STEPS] [--max-chunks K]\n");
    return 1;
  }
  static problem q;
  if (!read_problem(prob_path, &q)) return 1;

  lbm_throat_t h = NULL;
  int rc = lbm_throat_init(&q.p, &h);
  if (rc < 0) return fail("lbm_throat_init", rc);
  int status = 0;
  if (ckpt && file_exists(ckpt)) {
    rc = lbm_load(h, ckpt);
    if (rc < 0) {
      status = fail("lbm_load", rc);
      goto out;
    }
    fprintf(stderr, "lbm_drain: resumed from %s\n", ckpt);
  } else {
    rc = lbm_drain_begin(h, q.pc, q.n_pc, &q.conv);
    if (rc < 0) {
      status = fail("lbm_drain_begin", rc);
      goto out;
    }
  }

  int done = 0;
  long long chunks = 0;
  double S[MAX_PC];
  long long steps[MAX_PC];
  int pst[MAX_PC];
  lbm_drain_result r;
  memset(&r, 0, sizeof r);
  r.S = S;
  r.steps = steps;
  r.status = pst;
  while (!done) {
    if (max_chunks >= 0 && chunks >= max_chunks) {
      fprintf(stderr, "lbm_drain: stopped after %lld chunks\n", chunks);
      status = 3;
      goto out;
    }
    rc = lbm_drain_advance(h, chunk, &done);
    if (rc < 0) {
      status = fail("lbm_drain_advance", rc);
      goto out;
    }
    ++chunks;
    if (ckpt) {
      char tmp[4096];
      if (snprintf(tmp, sizeof tmp, "%s.tmp", ckpt) >= (int)sizeof tmp) {
        fprintf(stderr, "lbm_drain: checkpoint path too long\n");
        status = 1;
        goto out;
      }
      rc = lbm_save(h, tmp);
      if (rc < 0 || rename(tmp, ckpt) != 0) {
        status = rc < 0 ? fail("lbm_save", rc) : 2;
        if (rc >= 0) fprintf(stderr, "lbm_drain: cannot rename %s to %s\n", tmp, ckpt);
        goto out;
      }
    }
    rc = lbm_drain_get(h, q.n_pc, &r, &done);
    if (rc < 0) {
      status = fail("lbm_drain_get", rc);
      goto out;
    }
    fprintf(stderr, "lbm_drain: chunk %lld, %lld lattice steps so far\n", chunks, r.total_steps);
  }
  rc = lbm_drain_get(h, q.n_pc, &r, &done);
  if (rc < 0) {
    status = fail("lbm_drain_get", rc);
    goto out;
  }
  double mass[2], sw;
  rc = lbm_reduce(h, mass, &sw);
  if (rc < 0) {
    status = fail("lbm_reduce", rc);
    goto out;
  }
  printf("invaded_at %d\nn_bisect %d\ntotal_steps %lld\nfailed %d\n", r.invaded_at, r.n_bisect,
         r.total_steps, r.failed);
  printf("pce %.17g\npce_lo %.17g\npce_hi %.17g\n", r.pce, r.pce_lo, r.pce_hi);
  printf("S");
  for (int i = 0; i < q.n_pc; ++i) printf(" %.17g", S[i]);
  printf("\nsteps");
  for (int i = 0; i < q.n_pc; ++i) printf(" %lld", steps[i]);
  printf("\nstatus");
  for (int i = 0; i < q.n_pc; ++i) printf(" %d", pst[i]);
  printf("\nmass %.17g %.17g\nS_w %.17g\n", mass[0], mass[1], sw);
out:
  lbm_throat_free(h);
  return status;
}
