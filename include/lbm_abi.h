/*
 * lbm_abi.h -- C interface of the MI355X two-component Shan-Chen throat
 * drainage library.
 *
 * Method: Montella, Yuan, Chareyre, Gens, "A Hybrid multiphase model based on
 * lattice Boltzmann method direct simulations".  Each pore throat of a sphere
 * packing is a small subdomain (Sec. 2.2.2: a triangular prism whose three
 * walls pass through pairs of sphere centres, closed by inlet and outlet
 * sections) in which a two-component Shan-Chen lattice Boltzmann model runs
 * (Sec. 2.1, Eq. 1-5: D3Q19 BGK, moments, cohesion force, non-ideal
 * equation of state).  The inlet/outlet densities are stepped to raise the
 * capillary pressure; the entry capillary pressure p_c^e is the largest
 * pressure the throat holds before the non-wetting phase invades the pore
 * body (Sec. 2.2.2, definition of p_c^e).
 *
 * Conventions shared by every entry point:
 *  - Lattice units, dx = dt = 1.  Component 0 = wetting (w), 1 = non-wetting
 *    (nw).  Per-node arrays are laid out x fastest, then y, then z; population
 *    arrays are [component][direction][z][y][x].
 *  - D3Q19 direction order: 0 rest; 1..6 = +x,-x,+y,-y,+z,-z; 7..18 =
 *    (+1,+1,0) (-1,-1,0) (+1,-1,0) (-1,+1,0) (+1,0,+1) (-1,0,-1) (+1,0,-1)
 *    (-1,0,+1) (0,+1,+1) (0,-1,-1) (0,+1,-1) (0,-1,+1); opposite directions are
 *    adjacent (odd k <-> k+1).  Weights 1/3, 1/18, 1/36; c_s^2 = 1/3.
 *  - Node classes (voxelization, node (i,j,k) at integer coordinates): solid
 *    if (i-cx)^2 + (j-cy)^2 + (k-cz)^2 <= r^2 for any sphere (evaluated in
 *    FP64 term by term, no fused multiply-add), or, with a prism closure,
 *    if (i,j) lies outside the triangle of the three prism sphere centres;
 *    else an inlet bath node (z = 0) or outlet bath node (z = nz-1) when the
 *    z boundary is LBM_BC_RESERVOIR; else fluid.
 *  - Every pointer argument is a HOST pointer unless stated otherwise.  The
 *    caller owns all arrays it passes in and all output arrays; sizes are
 *    implied by the other arguments.  The library owns handles and the
 *    device memory behind them.
 *  - Errors: functions never abort or throw; they return a negative status,
 *    leave outputs untouched, and record a message for lbm_last_error().
 *    A positive status is a warning with valid outputs.
 *  - Device work runs on the handle's stream (lbm_params.stream, a
 *    hipStream_t, or the null stream).  Calls on one handle must not overlap
 *    from several host threads.
 */
#ifndef LBM_ABI_H
#define LBM_ABI_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define LBM_OK 0
#define LBM_EINVAL (-1)     /* invalid argument                            */
#define LBM_ENOMEM (-2)     /* device or host allocation failed / too big  */
#define LBM_EHIP (-3)       /* a HIP runtime call failed                    */
#define LBM_ENONFINITE (-4) /* the state became non-finite                  */
#define LBM_ESTATE (-5)     /* call not valid in the handle's state         */
#define LBM_EIO (-6)        /* a checkpoint file could not be written/read  */
#define LBM_WNOTCONV 1      /* a ramp point hit its step cap, or bisection
                               its run limit                                */
#define LBM_WPARTIAL 2      /* batch: some subdomains failed (see status)  */

/* boundary kinds, one per axis */
#define LBM_BC_PERIODIC 0
#define LBM_BC_WALLS 1      /* nodes beyond the box are solid              */
#define LBM_BC_RESERVOIR 2  /* z only: z = 0 and z = nz-1 are density baths */

/* node classes reported by lbm_get_types */
#define LBM_NODE_FLUID 0
#define LBM_NODE_SOLID 1
#define LBM_NODE_RES_IN 2
#define LBM_NODE_RES_OUT 3

/* per-ramp-point status */
#define LBM_PT_CONVERGED 0
#define LBM_PT_NOT_CONVERGED 1
#define LBM_PT_NONFINITE 2
#define LBM_PT_NOT_RUN 3    /* batch: the point was never reached        */

typedef struct {
  double c[3]; /* centre, lattice units */
  double r;    /* radius, lattice units */
} lbm_sphere;

/* Statement of one subdomain run (Sec. 2.1 and 2.2). */
typedef struct {
  int nx, ny, nz;            /* box size in nodes, each >= 3, product < 2^29,
                                nx, ny rounded up to multiples of 8 and 4:
                                product <= 9,418,786 (3-plane pull offsets)  */
  int bc[3];                 /* LBM_BC_* for x, y, z (RESERVOIR only for z)   */
  int n_spheres;             /* >= 0                                          */
  const lbm_sphere *spheres; /* [n_spheres], host                             */
  int prism;                 /* 1: solid outside the z-prism over 3 centres   */
  int prism_ids[3];          /* indices into spheres (used when prism = 1)    */
  double tau[2];             /* relaxation times (Eq. 1), each > 0.5          */
  double G;                  /* cohesion strength (Eq. 4-5)                   */
  double G_ads[2];           /* adhesion strength per component               */
  double rho_major;          /* majority density of a bulk phase, > 0         */
  double rho_minor;          /* minority density of a bulk phase, > 0         */
  double rho_in_nw;          /* nw density of the inlet bath, > 0             */
  double rho_out_w;          /* w density of the outlet bath, > 0             */
  const double *rho_init;    /* host [2][nz][ny][nx] initial densities, or
                                NULL: nw (rho_major) in z <= z_front, w above */
  int z_front;
  int probe[3];              /* pore-body probe node; probe[0] < 0: none      */
  void *stream;              /* hipStream_t or NULL                           */
} lbm_params;

/* Steady-state test and bisection of one drainage ramp. */
typedef struct {
  double tol;          /* stop when |S_w(t) - S_w(t - check_every)| < tol   */
  int check_every;     /* steps between saturation checks, >= 1             */
  long long max_steps; /* cap per ramp point (and per bisection run)        */
  double bisect_rel;   /* stop bisecting when (hi - lo)/hi <= bisect_rel     */
} lbm_conv;

/* Result of one drainage ramp.  S, steps and status point to caller arrays
 * of n_pc entries. */
typedef struct {
  double pce;          /* entry capillary pressure: midpoint of [lo, hi]   */
  double pce_lo;       /* largest pressure found stable                     */
  double pce_hi;       /* smallest pressure found invaded                   */
  int invaded_at;      /* first invaded ramp index, -1 if none              */
  int n_bisect;        /* bisection runs made                               */
  long long total_steps; /* lattice steps run, ramp plus bisection          */
  double *S;           /* [n_pc] wetting saturation at the end of each point */
  long long *steps;    /* [n_pc] steps used by each point                   */
  int *status;         /* [n_pc] LBM_PT_*                                   */
  int failed;          /* 1: the state became non-finite (batch only; a
                          single drain returns LBM_ENONFINITE instead): the
                          failing point and every later one carry
                          LBM_PT_NONFINITE and pce, pce_lo, pce_hi are NaN */
} lbm_drain_result;

typedef struct lbm_throat *lbm_throat_t;

/* Device-memory budget of the library's allocating calls, for callers that
 * share the GPU: with bytes > 0, lbm_throat_init, lbm_drain_throat,
 * lbm_drain_batch and lbm_place compute the device memory a call needs before allocating
 * anything (per subdomain: two population buffers of 152 bytes per padded
 * node, plus 25 bytes per node of masks, classes, densities and the node
 * list; two more population buffers for the ramp checkpoints of a drain) and
 * refuse a call that needs more than `bytes` with LBM_ENOMEM, having
 * allocated nothing.  0 (the default) sets no budget; calls are then refused
 * only when the device reports less free memory than they need.  Process
 * wide; takes effect for calls that start after it returns. */
int lbm_set_memory_budget(size_t bytes);

/* Create a subdomain: voxelize the geometry on the device, allocate two FP32
 * population buffers (2 x 152 bytes per node, nx and ny padded to multiples
 * of 8 and 4) and set the equilibrium state f = f_eq(rho_init, u = 0)
 * (Eq. 1-3).  Also per node: a 4-byte mask word, a 1-byte class and an
 * 8-byte density slot of the node-list path; per non-solid node an 8-byte
 * list entry.  *out receives the handle.
 * Errors: LBM_EINVAL (sizes < 3, tau <= 0.5, non-positive or non-finite
 * densities, bad prism ids, probe outside the fluid), LBM_ENOMEM, LBM_EHIP. */
int lbm_throat_init(const lbm_params *p, lbm_throat_t *out);

/* Release a handle and its device memory.  NULL is ignored. */
void lbm_throat_free(lbm_throat_t h);

/* Advance nsteps >= 0 time steps (Eq. 1: collide toward the component
 * equilibria with the cohesion (Eq. 4) and adhesion forces, then stream with
 * half-way bounce-back and bath re-imposition).  Asynchronous on the
 * handle's stream. */
int lbm_step(lbm_throat_t h, long long nsteps);

/* Wait for all work queued on the handle's stream. */
int lbm_sync(lbm_throat_t h);

/* Set the nw density of the inlet bath (takes effect from the next step). */
int lbm_set_rho_in(lbm_throat_t h, double rho_in_nw);

/* The inlet density that imposes capillary pressure pc: from Eq. 5 with the
 * minority density fixed, p_in - p_out = c_s^2 (1 + G rho_minor)
 * (rho_in - rho_out).  Returns NaN for a NULL handle. */
double lbm_rho_in_for_pc(lbm_throat_t h, double pc);

/* Node count and node classes (host uint8 [nz][ny][nx]). */
long long lbm_nodes(lbm_throat_t h);
int lbm_get_types(lbm_throat_t h, unsigned char *types);

/* Pre-collision populations at the current time, unshifted, as FP64:
 * host [2][19][nz][ny][nx]; zero on solid nodes. Synchronous. */
int lbm_get_populations(lbm_throat_t h, double *f);

/* Densities rho_w, rho_nw (Eq. 2): host [2][nz][ny][nx]; bath nodes hold the
 * imposed values, solid nodes zero. Synchronous. */
int lbm_get_density(lbm_throat_t h, double *rho);

/* The same read-back as lbm_get_density, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc): it calls no hipMalloc, hipFree or other allocating
 * routine.  The densities are staged in a fixed device array of 2^21 nodes x
 * 2 doubles (32 MiB, a 128^3 box), which each GPU the library runs on holds
 * from the first call until the process ends.  Boxes of more than 2^21 nodes
 * are refused with LBM_EINVAL (output untouched).  Every call on one GPU
 * stages through that GPU's one array: calls that overlap on one GPU (handles
 * on different streams or host threads) race and must be serialised by the
 * caller.  Synchronous on the handle's stream. */
int lbm_get_density_noalloc(lbm_throat_t h, double *rho);

/* FP64 reductions over fluid nodes: masses [2] (Eq. 2 summed) and the
 * wetting saturation S_w = mean of (phi + phi_b) / (2 phi_b) with
 * phi = (rho_w - rho_nw)/(rho_w + rho_nw), phi_b = (rho_major - rho_minor) /
 * (rho_major + rho_minor).  Either output may be NULL. Synchronous. */
int lbm_reduce(lbm_throat_t h, double *mass2, double *S_w);

/* 1 if rho_nw > rho_w at the probe node, else 0 (invasion test). */
int lbm_probe_invaded(lbm_throat_t h, int *invaded);

/* Drainage ramp (Sec. 2.2.2): for each pc[i] (strictly increasing), set the
 * inlet density for pc[i] and run until the saturation changes by less than
 * c->tol over c->check_every steps (or c->max_steps); record S_w.  At the
 * first invaded point, bisect between the last stable state and pc[i] on a
 * copy of the state until the bracket is within c->bisect_rel; the entry
 * pressure is reported as that bracket (Sec. 2.2.2: p_c^e is the maximum p_c
 * reached before invasion).  pc[0] must be > 0.  Bisection stops after 40
 * runs: a throat already invaded at pc[0] brackets from 0, where the
 * relative width may never shrink; its bracket is then reported as reached.
 * Synchronous.  Returns LBM_WNOTCONV if a point hit its cap or bisection its
 * run limit, LBM_ENONFINITE (outputs untouched) if the state became
 * non-finite. */
int lbm_drain_throat(lbm_throat_t h, const double *pc, int n_pc, const lbm_conv *c,
                     lbm_drain_result *out);

/* The same drainage ramp in resumable form.  lbm_drain_begin validates as
 * lbm_drain_throat does, keeps pc and c in the handle and starts the first
 * point; lbm_drain_advance runs it in whole chunks of c->check_every steps
 * until it ends or max_steps (>= 0) lattice steps have run in this call
 * (*done = 1 once the ramp has ended; done may be NULL); lbm_drain_get
 * copies the results so far into out, whose arrays hold n_pc entries (n_pc
 * must equal the ramp's; points not reached yet carry LBM_PT_NOT_RUN), and
 * sets *done.  Begin + advance to the end + get gives
 * lbm_drain_throat's results bit for bit, however the steps are split
 * between calls and whether or not the handle was saved and loaded between
 * them.  A non-finite state ends the ramp with LBM_ENONFINITE (lbm_drain_get
 * then reports failed = 1).  lbm_drain_advance and lbm_drain_get return
 * LBM_ESTATE on a handle with no ramp begun; all three are synchronous. */
int lbm_drain_begin(lbm_throat_t h, const double *pc, int n_pc, const lbm_conv *c);
int lbm_drain_advance(lbm_throat_t h, long long max_steps, int *done);
int lbm_drain_get(lbm_throat_t h, int n_pc, lbm_drain_result *out, int *done);

/* Checkpoint and resume (Sec. 2.2.2's ramp is a long sequence of steady
 * states).  lbm_save writes to the file at `path` (host byte order): the
 * subdomain's size, a hash of its node classes and its parameters; the inlet
 * density and the step count; the state of a ramp begun with
 * lbm_drain_begin (point, bracket, results so far, the run in progress);
 * the current populations (FP32, 152 bytes per padded node, ghost planes
 * included) and, while a ramp is running, its two checkpoints.
 * lbm_load reads such a file into a handle created with the same statement
 * (lbm_params; the file is refused with LBM_EINVAL, handle untouched, when
 * size, node classes or parameters differ) and restores all of it: stepping
 * or advancing the ramp then continues bit for bit as in the handle that was
 * saved.  Errors: LBM_EIO when the file cannot be opened, written or read
 * (a load that fails while reading the populations leaves the handle's
 * state undefined: load again or free it), LBM_ENOMEM, LBM_EHIP.
 * Synchronous. */
int lbm_save(lbm_throat_t h, const char *path);
int lbm_load(lbm_throat_t h, const char *path);

/* Summary of a batched drainage (optional output of lbm_drain_batch). */
typedef struct {
  int tx, ty, lz;           /* launch shape chosen by the autotuner          */
  int n_tiles;              /* live tiles of all subdomains in one launch    */
  long long replays;        /* graph replays (chunks of check_every steps)   */
  long long lattice_steps;  /* fused-step launches issued                    */
  long long node_updates;   /* sum over subdomains of active steps x nodes   */
  long long fluid_updates;  /* the same with fluid nodes only                */
  double wall_ms;           /* device time from the first to the last kernel */
} lbm_batch_info;

/* Batched drainage of n subdomains (Sec. 2.2.2: the throats are solved
 * independently): p[t] states subdomain t (each needs a probe node), pc is
 * host [n][n_pc] (each row positive and strictly increasing), out[t] receives the same
 * results as lbm_drain_throat would (bit for bit: the same kernels and the
 * same reduction order).  One fused-step launch covers the live tiles of all
 * running subdomains; the ramp and bisection decisions are taken on the
 * device between chunks of c->check_every steps (even), captured once as a
 * HIP graph and replayed until every subdomain is done.  The launch shape is
 * autotuned over the whole batch.  Device memory: 4 x 152 bytes per node
 * (two buffers and two ramp checkpoints) plus what lbm_throat_init holds per
 * subdomain.  Synchronous.  Returns
 * LBM_WNOTCONV if a point hit its cap, LBM_WPARTIAL if a subdomain became
 * non-finite: its result has failed = 1, NaN entry pressures and
 * LBM_PT_NONFINITE from the failing point on; the other subdomains are
 * complete and equal their single drains.  info may be NULL.
 * With LBM_BATCH_NO_GRAPH=1 in the environment the chunks are launched
 * kernel by kernel instead of replayed as a graph (for tracers that do not
 * follow graph launches); the results are the same bit for bit. */
int lbm_drain_batch(int n, const lbm_params *p, const double *pc, int n_pc, const lbm_conv *c,
                    lbm_drain_result *out, lbm_batch_info *info);

/* Time nsteps steps of the fused update with HIP events on the handle's
 * stream; *ms receives the elapsed milliseconds.  Synchronous. */
int lbm_time_steps(lbm_throat_t h, long long nsteps, double *ms);

/* Event timing of the fused-step launches made inside lbm_drain_throat:
 * HIP events bracket each chunk of back-to-back step launches on the
 * handle's stream.  Returns the accumulated milliseconds and launch count
 * (either output may be NULL); enable = 1 / 0 resets the totals and turns
 * timing on / off, enable = -1 only reads. */
int lbm_step_timer(lbm_throat_t h, int enable, double *total_ms, long long *launches);

/* Launch shape of the step: tile (tx, ty) in {(32, 4), (32, 8), (64, 4),
 * (16, 4), (16, 8), (8, 8)} marching a z-segment of lz (>= 1) planes in one
 * fused pass; 0 keeps the current value.  tx = LBM_SCHED_NODE_LIST selects
 * the node-list path instead (two passes over the non-solid nodes only, for
 * mostly solid subdomains; ty and lz are ignored and read back as 0).  All
 * shapes give bit-identical results. */
#define LBM_SCHED_NODE_LIST (-1)
int lbm_set_schedule(lbm_throat_t h, int tx, int ty, int lz);

/* Autotune the launch shape for this subdomain: time `trial_steps` steps
 * for every tile shape in increasing z-segment length (up to the first that
 * is 1.5x slower than the shape's best) and for the node list, time the
 * candidates within 1.25x of the best once more (each keeps its faster
 * time), keep the fastest and return it (outputs may be NULL).  The trials step the state forward with
 * alternating buffers, as a drain does, from a copy that is restored at the
 * end, so the state is unchanged; the copy takes one more population buffer
 * of device memory while tuning (LBM_ENOMEM if it cannot be had).
 * Synchronous. */
int lbm_autotune(lbm_throat_t h, int trial_steps, int *tx, int *ty, int *lz);
int lbm_get_schedule(lbm_throat_t h, int *tx, int *ty, int *lz);

/* Placement of the two population buffers.  The step time of large,
 * HBM-bound subdomains depends by several per cent on where the buffers lie
 * in physical device memory, which an allocation cannot ask for.  This call
 * times trial_steps steps (after 2 untimed ones) at the current launch shape
 * on the current buffer pair and on up to `tries` (0..8) newly allocated
 * pairs, each allocated while the earlier ones are still held; it keeps the
 * fastest pair and frees the others.  As in lbm_autotune the trials run from
 * a copy of the state that is put back into the kept pair, so the state is
 * unchanged bit for bit.  *ms_first and *ms_best (either may be NULL)
 * receive the per-step time of the original pair and of the kept one.
 * Device memory while it runs: one population buffer for the copy plus two
 * per try (LBM_ENOMEM if the memory budget refuses that; a try whose
 * allocation fails ends the search without error).  Synchronous. */
int lbm_place(lbm_throat_t h, int tries, int trial_steps, double *ms_first, double *ms_best);

/* Stream-copy probe of the achievable HBM bandwidth (the measured roofline
 * denominator beside the 8 TB/s specification): copies `bytes` (>= 1 MiB)
 * between two device buffers `reps` times on the null stream and returns the
 * read + write rate in GB/s.  Allocates and frees 2 x bytes of device memory.
 * Synchronous. */
int lbm_bw_probe(size_t bytes, int reps, double *gbps);

/* Message of the last error on the calling thread ("" if none). */
const char *lbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
