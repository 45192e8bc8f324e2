// network.cpp -- quasi-static drainage of a pore network from per-throat
// entry pressures, with trapping of wetting regions cut off from the outlet
// (rules in lbm_network.h).  Host code: a binary heap of candidate throats
// keyed by (entry pressure, throat index), and after every invasion one
// traversal from the outlet over wetting pores.
#include <cmath>
#include <queue>
#include <tuple>
#include <vector>

#include "lbm_abi.h"
#include "lbm_handle.h"
#include "lbm_network.h"

using lbmh::set_err;

namespace {

struct Cand {
  double pce;
  int t, v;
  bool operator>(const Cand &o) const { return pce > o.pce || (pce == o.pce && t > o.t); }
};

}  // namespace

extern "C" int lbm_network_drain(int n_pores, const double *pore_vol, int n_throats,
                                 const int *throats, const double *pce, int n_p,
                                 const double *pressures, double *sw, int *invaded_at,
                                 int *state) {
  if (n_pores < 1 || n_throats < 0 || n_p < 1 || !pore_vol || (n_throats > 0 && (!throats || !pce)) ||
      !pressures || !sw || !invaded_at || !state) {
    set_err("lbm_network_drain: bad sizes or NULL arrays");
    return LBM_EINVAL;
  }
  double total = 0.0;
  for (int p = 0; p < n_pores; ++p) {
    if (!std::isfinite(pore_vol[p]) || pore_vol[p] < 0) {
      set_err("lbm_network_drain: pore %d has volume %g", p, pore_vol[p]);
      return LBM_ENONFINITE;
    }
    total += pore_vol[p];
  }
  if (!(total > 0)) {
    set_err("lbm_network_drain: the total void volume must be positive");
    return LBM_EINVAL;
  }
  for (int i = 0; i < n_p; ++i) {
    if (!std::isfinite(pressures[i]) || (i > 0 && !(pressures[i] > pressures[i - 1]))) {
      set_err("lbm_network_drain: pressures must be finite and strictly increasing");
      return LBM_EINVAL;
    }
  }
  // adjacency (compressed rows) and the pores that open onto the outlet
  std::vector<int> deg(n_pores + 1, 0), outlet_pores;
  for (int t = 0; t < n_throats; ++t) {
    const int a = throats[2 * t], b = throats[2 * t + 1];
    if (a < LBM_NET_OUTLET || b < LBM_NET_OUTLET || a >= n_pores || b >= n_pores || (a < 0 && b < 0)) {
      set_err("lbm_network_drain: throat %d joins %d and %d", t, a, b);
      return LBM_EINVAL;
    }
    if (std::isnan(pce[t]) || pce[t] == -INFINITY) {
      set_err("lbm_network_drain: throat %d has entry pressure %g", t, pce[t]);
      return LBM_ENONFINITE;
    }
    if (a >= 0) ++deg[a + 1];
    if (b >= 0) ++deg[b + 1];
    if (a == LBM_NET_OUTLET) outlet_pores.push_back(b);
    if (b == LBM_NET_OUTLET) outlet_pores.push_back(a);
  }
  for (int p = 0; p < n_pores; ++p) deg[p + 1] += deg[p];
  std::vector<int> nb(deg[n_pores]), nt(deg[n_pores]), fill(deg.begin(), deg.end() - 1);
  for (int t = 0; t < n_throats; ++t) {
    const int a = throats[2 * t], b = throats[2 * t + 1];
    if (a >= 0) {
      nb[fill[a]] = b;
      nt[fill[a]++] = t;
    }
    if (b >= 0) {
      nb[fill[b]] = a;
      nt[fill[b]++] = t;
    }
  }

  std::vector<int> st(n_pores, LBM_NET_WETTING), inv(n_pores, -1), mark(n_pores, 0), stack;
  int stamp = 0;
  auto update_trapping = [&]() {
    ++stamp;
    stack.clear();
    for (int p : outlet_pores)
      if (st[p] == LBM_NET_WETTING && mark[p] != stamp) {
        mark[p] = stamp;
        stack.push_back(p);
      }
    while (!stack.empty()) {
      const int p = stack.back();
      stack.pop_back();
      for (int j = deg[p]; j < deg[p + 1]; ++j) {
        const int q = nb[j];
        if (q >= 0 && st[q] == LBM_NET_WETTING && mark[q] != stamp) {
          mark[q] = stamp;
          stack.push_back(q);
        }
      }
    }
    for (int p = 0; p < n_pores; ++p)
      if (st[p] == LBM_NET_WETTING && mark[p] != stamp) st[p] = LBM_NET_TRAPPED;
  };

  std::priority_queue<Cand, std::vector<Cand>, std::greater<Cand>> heap;
  for (int t = 0; t < n_throats; ++t) {
    const int a = throats[2 * t], b = throats[2 * t + 1];
    if (a == LBM_NET_INLET) heap.push(Cand{pce[t], t, b});
    if (b == LBM_NET_INLET) heap.push(Cand{pce[t], t, a});
  }
  for (int i = 0; i < n_p; ++i) {
    while (!heap.empty() && heap.top().pce <= pressures[i]) {
      const Cand c = heap.top();
      heap.pop();
      if (st[c.v] != LBM_NET_WETTING) continue;  // invaded or trapped since it was queued
      st[c.v] = LBM_NET_INVADED;
      inv[c.v] = i;
      for (int j = deg[c.v]; j < deg[c.v + 1]; ++j) {
        const int q = nb[j];
        if (q >= 0 && st[q] == LBM_NET_WETTING) heap.push(Cand{pce[nt[j]], nt[j], q});
      }
      update_trapping();
    }
    double wet = 0.0;
    for (int p = 0; p < n_pores; ++p)
      if (st[p] != LBM_NET_INVADED) wet += pore_vol[p];
    sw[i] = wet / total;
  }
  for (int p = 0; p < n_pores; ++p) {
    invaded_at[p] = inv[p];
    state[p] = st[p];
  }
  return LBM_OK;
}
