/* lbm_network.h -- quasi-static drainage of a pore network.
 *
 * The hybrid method decomposes the pore space of a packing into pore bodies
 * (the tetrahedra of a regular triangulation, Sec. 2.2.1) joined by pore
 * throats (their facets), solves each throat with the LBM for its entry
 * capillary pressure (Sec. 2.2.2), and assembles the drainage of the whole
 * sample from those entry pressures: the non-wetting phase passes a throat
 * when the capillary pressure exceeds the throat's entry pressure, and
 * wetting regions cut off from the outlet keep their fluid (Sec. 3.1.1).
 *
 * Rules, applied for each capillary pressure p_i in increasing order:
 *   - candidates are throats joining the inlet reservoir or an invaded pore
 *     to a wetting pore, with entry pressure <= p_i;
 *   - the candidate with the smallest (entry pressure, throat index) is
 *     invaded first, then the next, until none is left at p_i;
 *   - after every invasion, wetting pores no longer connected to the outlet
 *     reservoir through wetting pores become trapped and are never invaded;
 *   - the wetting saturation after p_i is the void volume of wetting and
 *     trapped pores over the total void volume (summed in pore order).
 * Every pore starts wetting.  Host code; no device memory is used.
 *
 * Status codes and lbm_last_error() as in lbm_abi.h.
 */
#ifndef LBM_NETWORK_H
#define LBM_NETWORK_H

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_NET_INLET (-1)   /* throat end: the non-wetting reservoir */
#define LBM_NET_OUTLET (-2)  /* throat end: the wetting reservoir     */
#define LBM_NET_WETTING 0
#define LBM_NET_INVADED 1
#define LBM_NET_TRAPPED 2

/* n_pores >= 1 pores with void volumes pore_vol [n_pores] (>= 0, positive
 * sum); n_throats throats with ends throats [n_throats][2] (pore index or
 * LBM_NET_INLET / LBM_NET_OUTLET, at least one end a pore) and entry
 * pressures pce [n_throats] (finite or +infinity: never passed); n_p
 * capillary pressures, strictly increasing.  Outputs (host, caller-owned):
 * sw [n_p]; invaded_at [n_pores] (index of the pressure at which the pore was
 * invaded, -1 if never); state [n_pores] (LBM_NET_*).  Returns LBM_OK or
 * LBM_EINVAL / LBM_ENONFINITE with nothing written. */
int lbm_network_drain(int n_pores, const double *pore_vol, int n_throats, const int *throats,
                      const double *pce, int n_p, const double *pressures, double *sw,
                      int *invaded_at, int *state);

#ifdef __cplusplus
}
#endif

#endif
