"""FP64 reference of the learned entry-pressure surrogate (test infrastructure).

TEST INFRASTRUCTURE ONLY: imported by the tests and never by the product
path.  Plain numpy in float64, written from the definitions below, sharing no
code with the HIP library.

What it computes.  The paper solves every pore throat with a full LBM run
(Sec. 2.2.2) and names that cost as the obstacle (Sec. 4); the surrogate maps a
throat's geometry to its entry capillary pressure and drainage curve so that
the LBM runs only where an ensemble of networks disagrees.

* Descriptor (80 values per throat).  With the three throat spheres (the
  prism spheres, in the order given) and the fourth (downstream) sphere,
  rbar = mean radius of the three throat spheres and c = centroid of their
  centres:
    - 4 radii / rbar (throat spheres first, then the fourth);
    - 12 values (centre - c) / rbar, x y z per sphere in the same order;
    - 64 occupancy values: the box is sampled at 32^3 points
      x_i = (i + 0.5) * nx / 32 - 0.5 (likewise y, z); a point is solid if it
      lies in a sphere (|p - centre|^2 <= r^2) or outside the prism over the
      triangle of throat-sphere centres; the solid fraction of every 8^3 block
      of samples gives a 4^3 grid, x fastest.
* Network, per ensemble member: 80 -> 256 -> 256 -> 256 -> 17, SiLU after
  each hidden layer (silu(z) = z / (1 + exp(-z))), linear output.  Weights
  W_l have shape [out][in]; a member's parameters are the flat concatenation
  W_1, b_1, W_2, b_2, W_3, b_3, W_4, b_4 (156,689 values).
* Loss: mean squared error over the batch and the 17 outputs, on standardised
  targets.
* Adam (Kingma & Ba 2015) with bias correction: m = b1 m + (1 - b1) g,
  v = b2 v + (1 - b2) g^2, w -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
* Ensemble: mean and population standard deviation over members; a throat
  falls back to the LBM when std(p) > threshold * |mean(p)| for output 0.
* Targets: output 0 is p_c^e times the throat's MS-P entry radius (computed
  by the HIP library from the three throat circles; a throat without one is
  left out), outputs 1-16 the ramp's saturations.
* Opening radius (kept as a geometric reference): the circle in the prism's
  cross-section (xy) tangent from outside to the three throat-sphere
  circles, found by a root finder from the centroid.
"""
import numpy as np

LAYERS = (80, 256, 256, 256, 17)
N_OCC = 32       # occupancy samples per axis
POOL = 8         # samples per pooled cell and axis
N_FEAT = 80
N_OUT = 17


def n_params(layers=LAYERS):
    return sum(layers[i + 1] * layers[i] + layers[i + 1] for i in range(len(layers) - 1))


def unpack(flat, layers=LAYERS):
    """Flat member parameters -> [(W [out][in], b [out]), ...] (views)."""
    out, o = [], 0
    for i in range(len(layers) - 1):
        nin, nout = layers[i], layers[i + 1]
        W = flat[o:o + nout * nin].reshape(nout, nin)
        o += nout * nin
        b = flat[o:o + nout]
        o += nout
        out.append((W, b))
    assert o == flat.size
    return out


def silu(z):
    with np.errstate(over="ignore"):
        return z / (1.0 + np.exp(-z))


def dsilu(z):
    """d silu / dz = s (1 + z (1 - s)) with s the logistic function."""
    with np.errstate(over="ignore"):
        s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(flat, X, layers=LAYERS):
    """Outputs [B][17] and the cache (layer inputs, pre-activations)."""
    params = unpack(np.asarray(flat, dtype=np.float64), layers)
    a = np.asarray(X, dtype=np.float64)
    inputs, pre = [], []
    for li, (W, b) in enumerate(params):
        inputs.append(a)
        z = a @ W.T + b
        pre.append(z)
        a = silu(z) if li < len(params) - 1 else z
    return a, (inputs, pre)


def mse(Y, T):
    return float(np.mean((Y - T) ** 2))


def backward(flat, cache, Y, T, layers=LAYERS):
    """Gradient of mse(Y, T) with respect to the flat parameters."""
    params = unpack(np.asarray(flat, dtype=np.float64), layers)
    inputs, pre = cache
    d = 2.0 * (Y - T) / Y.size          # dL/dz of the output layer
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        grads[li] = (d.T @ inputs[li], d.sum(axis=0))
        if li > 0:
            d = (d @ W) * dsilu(pre[li - 1])
    return np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])


def adam(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1) of flat arrays, in place."""
    m *= b1
    m += (1.0 - b1) * g
    v *= b2
    v += (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    w -= lr * mh / (np.sqrt(vh) + eps)


def standardise_stats(A):
    """Column means and standard deviations (population); a column with
    std < 1e-12 gets std 1."""
    mu = A.mean(axis=0)
    sd = A.std(axis=0)
    sd = np.where(sd < 1e-12, 1.0, sd)
    return mu, sd


def train(members, X, T, order, batch, lr_max, epochs, lr_min_frac=0.0):
    """Train every member with Adam on standardised data.

    members: list of flat parameter arrays (updated in place).  order:
    int array [epochs][n_members][n] of sample indices (the member's
    bootstrap resample, shuffled per epoch).  Minibatches are consecutive
    slices of `batch` indices (the last one may be short).  The learning rate
    follows a cosine from lr_max at step 0 to lr_min_frac * lr_max after the
    last step.  Returns (X stats, T stats, per-epoch mean loss over members)."""
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    mx, sx = standardise_stats(X)
    mt, st = standardise_stats(T)
    Xs = (X - mx) / sx
    Ts = (T - mt) / st
    n = X.shape[0]
    per_epoch = (n + batch - 1) // batch
    total = epochs * per_epoch
    state = [(np.zeros_like(w), np.zeros_like(w)) for w in members]
    hist = []
    for e in range(epochs):
        losses = []
        for z, w in enumerate(members):
            m, v = state[z]
            le = 0.0
            for s in range(per_epoch):
                idx = order[e, z, s * batch:(s + 1) * batch]
                Y, cache = forward(w, Xs[idx])
                le += mse(Y, Ts[idx])
                g = backward(w, cache, Y, Ts[idx])
                step = e * per_epoch + s
                lr = lr_schedule(lr_max, lr_min_frac, step, total)
                adam(w, g, m, v, step + 1, lr)
            losses.append(le / per_epoch)
        hist.append(float(np.mean(losses)))
    return (mx, sx), (mt, st), hist


def lr_schedule(lr_max, lr_min_frac, step, total):
    """Cosine decay from lr_max (step 0) to lr_min_frac * lr_max (step total)."""
    c = 0.5 * (1.0 + np.cos(np.pi * step / max(total, 1)))
    return lr_max * (lr_min_frac + (1.0 - lr_min_frac) * c)


def predict(members, xstats, tstats, X):
    """Ensemble mean and population std of the de-standardised outputs."""
    Xs = (np.asarray(X, dtype=np.float64) - xstats[0]) / xstats[1]
    Ys = np.stack([forward(w, Xs)[0] * tstats[1] + tstats[0] for w in members])
    return Ys.mean(axis=0), Ys.std(axis=0)


def fallback(mean, std, threshold):
    return std[:, 0] > threshold * np.abs(mean[:, 0])


def _edge(P, Q, x, y):
    return (Q[0] - P[0]) * (y - P[1]) - (Q[1] - P[1]) * (x - P[0])


def descriptor(spheres, nx, ny, nz, prism_ids=(0, 1, 2)):
    """The 80 descriptor values of one four-sphere throat (see the header)."""
    S = np.asarray(spheres, dtype=np.float64)
    assert S.shape == (4, 4)
    ids = list(prism_ids) + [i for i in range(4) if i not in prism_ids]
    S = S[ids]
    rbar = S[:3, 3].mean()
    c = S[:3, :3].mean(axis=0)
    geo = np.concatenate([S[:, 3] / rbar, ((S[:, :3] - c) / rbar).ravel()])
    # sample points, z slowest
    ii = np.arange(N_OCC, dtype=np.float64)
    px = (ii + 0.5) * nx / N_OCC - 0.5
    py = (ii + 0.5) * ny / N_OCC - 0.5
    pz = (ii + 0.5) * nz / N_OCC - 0.5
    Z, Y, X = np.meshgrid(pz, py, px, indexing="ij")
    solid = np.zeros(X.shape, dtype=bool)
    for s in S:
        dx, dy, dz = X - s[0], Y - s[1], Z - s[2]
        solid |= dx * dx + dy * dy + dz * dz <= s[3] * s[3]
    A, B, C = S[0], S[1], S[2]
    o = _edge(A, B, C[0], C[1])
    e1, e2, e3 = _edge(A, B, X, Y), _edge(B, C, X, Y), _edge(C, A, X, Y)
    inside = (e1 >= 0) & (e2 >= 0) & (e3 >= 0) if o > 0 else (e1 <= 0) & (e2 <= 0) & (e3 <= 0)
    solid |= ~inside
    k = N_OCC // POOL
    occ = solid.reshape(k, POOL, k, POOL, k, POOL).sum(axis=(1, 3, 5)) / float(POOL ** 3)
    return np.concatenate([geo, occ.ravel()])


def opening_radius(spheres, prism_ids=(0, 1, 2)):
    """Radius of the circle in the xy-plane tangent from outside to the three
    circles (x_i, y_i, R_i) of the throat spheres: |c - P_i| = r + R_i."""
    from scipy.optimize import fsolve
    S = np.asarray(spheres, dtype=np.float64)[list(prism_ids)]

    def res(v):
        return [np.hypot(v[0] - S[i, 0], v[1] - S[i, 1]) - v[2] - S[i, 3] for i in range(3)]

    c = S[:, :2].mean(axis=0)
    r0 = max(np.hypot(*(S[:, :2] - c).T).mean() - S[:, 3].mean(), 1e-3)
    v, info, ok, _ = fsolve(res, [c[0], c[1], r0], full_output=True, xtol=1e-13)
    return float(v[2]) if ok == 1 else float("nan")
