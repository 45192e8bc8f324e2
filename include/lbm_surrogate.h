/* lbm_surrogate.h -- learned entry-pressure surrogate with LBM fallback.
 *
 * The hybrid method solves every pore throat with its own LBM drainage run
 * (Sec. 2.2.2) and identifies that cost as what limits it (Sec. 4).  This
 * part of the library maps the geometry of a four-sphere throat to its entry
 * capillary pressure p_c^e and a 16-point drainage curve with an ensemble of
 * small networks trained on throats that lbm_drain_batch itself solved, and
 * runs the LBM only for throats on which the ensemble disagrees.
 *
 * Model (fixed): per member an MLP 80 -> 256 -> 256 -> 256 -> 17 with SiLU
 * after the hidden layers.  Parameters of one member are the flat FP32 array
 * W1 b1 W2 b2 W3 b3 W4 b4 (W_l row-major [out][in]), LBM_SG_NPARAM values.
 * Products run on the matrix cores in BF16 with FP32 accumulation; master
 * weights, Adam moments and biases stay FP32; statistics are FP64.
 *
 * Descriptor (80 values per throat; lbm_surrogate_describe): with rbar the
 * mean radius of the three throat (prism) spheres and c the centroid of
 * their centres: the 4 radii / rbar (throat spheres in prism_ids order, then
 * the fourth), the 12 coordinates (centre - c) / rbar in the same order, and
 * the solid fraction of the 4^3 cells of 8^3 samples of a 32^3 sampling of
 * the box (sample i of an axis of n nodes at (i + 0.5) n / 32 - 0.5; solid
 * means inside a sphere or outside the prism, as the voxelizer decides).
 *
 * Targets (17 values per throat): p_c^e * r_msp (lattice pressure times
 * lattice length, in units of the interfacial tension of the model), then
 * the wetting saturation at the 16 points of the drainage ramp the training
 * data were produced with.  r_msp is the Mayer-Stowe-Princen corner-meniscus
 * radius at entry of the throat's cross-section (Sec. 1 of the paper names
 * the method): the plane of the three throat-sphere centres, the triangle of
 * centres (the prism's walls) minus the three circles, and the root r of the
 * force balance A_n = r (L_nw + L_ns) of a perfectly wetting solid, whose
 * entry pressure is gamma / r (lbm_surrogate_describe returns it).  So
 * p_c^e * r_msp is about gamma, and the network learns how each throat
 * departs from that estimate.
 *
 * Conventions as in lbm_abi.h: status codes LBM_*, host arrays owned by the
 * caller, lbm_last_error() for the message of the last failure.
 */
#ifndef LBM_SURROGATE_H
#define LBM_SURROGATE_H

#include "lbm_abi.h"

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_SG_NFEAT 80
#define LBM_SG_NOUT 17
#define LBM_SG_NCURVE 16
#define LBM_SG_NPARAM 156689
#define LBM_SG_MAX_BATCH 4096
#define LBM_SG_MAX_MEMBERS 16

typedef struct lbm_surrogate *lbm_surrogate_t;

typedef struct {
  int epochs;            /* passes over the training set (>= 1)                 */
  int batch;             /* minibatch size, 1 .. LBM_SG_MAX_BATCH               */
  double lr;             /* peak Adam step; cosine decay to lr * lr_min_frac    */
  double lr_min_frac;    /* in [0, 1]                                           */
  double beta1, beta2;   /* Adam moment decays, e.g. 0.9 and 0.999              */
  double eps;            /* Adam denominator guard, e.g. 1e-8                   */
  unsigned long long seed; /* sample order when no order is given               */
  int bootstrap;         /* 1: every member draws its own resample of the set   */
} lbm_sg_train_cfg;

typedef struct {
  int n_fallback;        /* throats handed to the LBM                          */
  double describe_ms;    /* descriptor kernels                                 */
  double predict_ms;     /* standardise + ensemble forward + statistics         */
  double lbm_ms;         /* fallback lbm_drain_batch wall time (0 if none)      */
  lbm_batch_info lbm;    /* its summary (zeroed if none)                        */
} lbm_sg_info;

/* New ensemble of `members` (1 .. LBM_SG_MAX_MEMBERS) networks, weights drawn
 * uniform in +-sqrt(3 / fan_in) from SplitMix64 streams of `seed`, biases 0,
 * no standardisation statistics yet.  stream: hipStream_t or NULL (own). */
int lbm_surrogate_create(int members, unsigned long long seed, void *stream, lbm_surrogate_t *out);
void lbm_surrogate_free(lbm_surrogate_t m); /* NULL is ignored */
int lbm_surrogate_members(lbm_surrogate_t m);

/* Copy one member's flat FP32 parameters in or out (host [LBM_SG_NPARAM]).
 * Setting parameters resets that member's Adam state. */
int lbm_surrogate_set_params(lbm_surrogate_t m, int member, const float *w);
int lbm_surrogate_get_params(lbm_surrogate_t m, int member, float *w);

/* Standardisation statistics: feature means/stds [80], target means/stds [17]
 * (host FP64).  lbm_surrogate_train sets them from its data. */
int lbm_surrogate_set_stats(lbm_surrogate_t m, const double *xmu, const double *xsd,
                            const double *tmu, const double *tsd);
int lbm_surrogate_get_stats(lbm_surrogate_t m, double *xmu, double *xsd, double *tmu, double *tsd);

/* Descriptors of n throats (each exactly 4 spheres with a prism closure) on
 * the GPU; feat: host [n][80]; r_msp: host [n] MS-P corner-meniscus radii at
 * entry in lattice units (NaN where the balance has no root before the
 * menisci meet), or NULL. */
int lbm_surrogate_describe(int n, const lbm_params *p, double *feat, double *r_msp);

/* Raw ensemble forward on standardised inputs xs (host [n][80]): y host
 * [members][n][17] FP32, standardised outputs. */
int lbm_surrogate_forward(lbm_surrogate_t m, int n, const double *xs, float *y);

/* Gradient of the mean squared error over one batch of standardised inputs
 * and targets (host [n][80], [n][17], n <= LBM_SG_MAX_BATCH), the same batch
 * for every member: grad host [members][LBM_SG_NPARAM], loss host [members].
 * Parameters are not changed. */
int lbm_surrogate_grad(lbm_surrogate_t m, int n, const double *xs, const double *ts, float *grad,
                       double *loss);

/* Train every member with Adam on raw features and targets (host [n][80],
 * [n][17]); sets the statistics from the data first.  order: host int
 * [epochs][members][n] sample indices (each member's resample, shuffled per
 * epoch; minibatches are consecutive slices of cfg->batch), or NULL to draw
 * them from cfg->seed.  loss_hist: host [epochs] mean training loss over
 * members, or NULL.  Synchronous. */
int lbm_surrogate_train(lbm_surrogate_t m, int n, const double *feat, const double *target,
                        const lbm_sg_train_cfg *cfg, const int *order, double *loss_hist);

/* Ensemble mean and population std of the de-standardised outputs for raw
 * features (host [n][80] -> [n][17] each).  Needs statistics. */
int lbm_surrogate_predict(lbm_surrogate_t m, int n, const double *feat, double *mean, double *std);

/* Entry pressure of n throats: describe, predict, and where the ensemble std
 * of output 0 exceeds threshold * |mean| (and run_fallback is 1) drain the
 * throat with lbm_drain_batch over pc (host [n][n_pc], n_pc = 16) and c, and
 * take its result.  The network's p_c^e is output 0 divided by r_msp; a
 * throat without an MS-P radius counts as disagreeing (drained by the LBM
 * when run_fallback is 1, NaN otherwise).
 * pce [n], curve [n][16], pce_std [n] (ensemble std of p_c^e; 0 where the
 * LBM answered), used_fallback [n] are host outputs: 0 network answer, 1 LBM
 * answer, 2 the LBM drain of the throat became non-finite (pce and pce_std
 * NaN; the call then returns LBM_WPARTIAL); info may be NULL.
 * Returns the fallback batch's warning code if any. */
int lbm_surrogate_pce(lbm_surrogate_t m, int n, const lbm_params *p, const double *pc, int n_pc,
                      const lbm_conv *c, double threshold, int run_fallback, double *pce,
                      double *curve, double *pce_std, int *used_fallback, lbm_sg_info *info);

#ifdef __cplusplus
}
#endif

#endif
