"""Reference of the pore-network drainage assembly (test infrastructure).

TEST INFRASTRUCTURE ONLY: used by the tests, never by the product path.
Plain Python over lists and sets, written from the rules below; it shares no
code with the native implementation.

Rules (Sec. 2.2.2 and Sec. 3.1.1 of the paper: the non-wetting phase passes a
throat when the capillary pressure exceeds the throat's entry pressure;
disconnected wetting regions keep their fluid; drainage is quasi-static and
pressure-controlled):

* every pore starts wetting (W);
* the capillary pressures p_0 < p_1 < ... are applied in order; at p_i the
  candidate throats are those joining the inlet reservoir or a non-wetting
  (N) pore to a W pore, with entry pressure <= p_i;
* candidates are invaded one at a time, the one with the smallest (entry
  pressure, throat index) first: the W pore becomes N;
* after each invasion, every W pore that is no longer connected to the outlet
  reservoir through W pores becomes trapped (T) and is never invaded;
* the wetting saturation after step i is the void volume of W and T pores
  over the total void volume.

Throat ends are pore indices, or -1 for the inlet (non-wetting) reservoir and
-2 for the outlet (wetting) reservoir.
"""
W, N, T = 0, 1, 2
INLET, OUTLET = -1, -2


def _update_trapping(state, adj, outlet_pores):
    reach = set()
    stack = [p for p in outlet_pores if state[p] == W]
    reach.update(stack)
    while stack:
        p = stack.pop()
        for q, _ in adj[p]:
            if q >= 0 and state[q] == W and q not in reach:
                reach.add(q)
                stack.append(q)
    for p in range(len(state)):
        if state[p] == W and p not in reach:
            state[p] = T


def drain(pore_vol, throats, pce, pressures):
    """Returns (wetting saturation per pressure, pressure index at which each
    pore was invaded or -1, final state per pore)."""
    n = len(pore_vol)
    adj = [[] for _ in range(n)]
    outlet_pores = []
    for t, (a, b) in enumerate(throats):
        a, b = int(a), int(b)
        if a >= 0:
            adj[a].append((b, t))
        if b >= 0:
            adj[b].append((a, t))
        if a == OUTLET and b >= 0:
            outlet_pores.append(b)
        if b == OUTLET and a >= 0:
            outlet_pores.append(a)
    state = [W] * n
    invaded_at = [-1] * n
    total = float(sum(pore_vol))
    sw = []
    for i, p in enumerate(pressures):
        while True:
            best = None
            for t, (a, b) in enumerate(throats):
                a, b = int(a), int(b)
                if pce[t] > p:
                    continue
                for u, v in ((a, b), (b, a)):
                    if v >= 0 and state[v] == W and (u == INLET or (u >= 0 and state[u] == N)):
                        cand = (pce[t], t, v)
                        if best is None or cand[:2] < best[:2]:
                            best = cand
            if best is None:
                break
            v = best[2]
            state[v] = N
            invaded_at[v] = i
            _update_trapping(state, adj, outlet_pores)
        sw.append(sum(pore_vol[q] for q in range(n) if state[q] != N) / total)
    return sw, invaded_at, state
