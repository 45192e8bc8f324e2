"""Hand-unrolled two-component Shan-Chen D3Q19 step on a tiny lattice.

An independent second implementation used only to check the oracle by brute
force: every direction is written out by hand (no loop over directions, no
shared tables), in numpy whole-array form.  Paper: Eq. 1 (BGK collide then
stream), Eq. 2-3 (moments), Eq. 4 (cohesion, read with D3Q19 weights and
Psi = rho), adhesion toward solid nodes, velocity-shift forcing of the cited
Shan-Chen model, half-way bounce-back, equilibrium baths on the z planes.

The population arrays are f[c][k] with shape (nz, ny, nx).
Node classes: 0 fluid, 1 solid, 2 inlet bath (z = 0), 3 outlet bath (z = nz-1).
"""
import numpy as np

W0, W1, W2 = 1.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0


def _shift(a, dx, dy, dz, periodic, fill):
    """b[z, y, x] = a[z + dz, y + dy, x + dx]; wraps on periodic axes,
    `fill` beyond the box otherwise."""
    out = a
    for axis, d, per in ((2, dx, periodic[0]), (1, dy, periodic[1]), (0, dz, periodic[2])):
        if d == 0:
            continue
        if per:
            out = np.roll(out, -d, axis=axis)
        else:
            rolled = np.roll(out, -d, axis=axis)
            idx = [slice(None)] * 3
            idx[axis] = slice(-1, None) if d > 0 else slice(0, 1)
            rolled[tuple(idx)] = fill
            out = rolled
    return out


def step(f, types, P, periodic):
    """One step.  f: array [2][19][nz][ny][nx]; P: dict with tau (2), G,
    G_ads (2), rho_major, rho_minor, rho_in_nw, rho_out_w."""
    fluid = types == 0
    solid = types == 1
    rin = types == 2
    rout = types == 3
    tau = P["tau"]
    G = P["G"]
    Ga = P["G_ads"]

    def res_rho(c):
        r = np.zeros(types.shape)
        if c == 0:
            r[rin] = P["rho_minor"]
            r[rout] = P["rho_out_w"]
        else:
            r[rin] = P["rho_in_nw"]
            r[rout] = P["rho_minor"]
        return r

    rho = []
    jx = []
    jy = []
    jz = []
    for c in (0, 1):
        g = f[c]
        r = (g[0] + g[1] + g[2] + g[3] + g[4] + g[5] + g[6] + g[7] + g[8] + g[9] + g[10]
             + g[11] + g[12] + g[13] + g[14] + g[15] + g[16] + g[17] + g[18])
        x = g[1] - g[2] + g[7] - g[8] + g[9] - g[10] + g[11] - g[12] + g[13] - g[14]
        y = g[3] - g[4] + g[7] - g[8] - g[9] + g[10] + g[15] - g[16] + g[17] - g[18]
        z = g[5] - g[6] + g[11] - g[12] - g[13] + g[14] + g[15] - g[16] - g[17] + g[18]
        r = np.where(fluid, r, res_rho(c))
        rho.append(r)
        jx.append(np.where(fluid, x, 0.0))
        jy.append(np.where(fluid, y, 0.0))
        jz.append(np.where(fluid, z, 0.0))

    def sh(a, dx, dy, dz, fill):
        return _shift(a, dx, dy, dz, periodic, fill)

    # density seen by the interaction sums: zero on solids and beyond walls
    seen = [np.where(solid, 0.0, rho[0]), np.where(solid, 0.0, rho[1])]
    s = solid.astype(np.float64)

    def grad(a, fill):
        gx = (W1 * (sh(a, 1, 0, 0, fill) - sh(a, -1, 0, 0, fill))
              + W2 * (sh(a, 1, 1, 0, fill) - sh(a, -1, -1, 0, fill)
                      + sh(a, 1, -1, 0, fill) - sh(a, -1, 1, 0, fill)
                      + sh(a, 1, 0, 1, fill) - sh(a, -1, 0, -1, fill)
                      + sh(a, 1, 0, -1, fill) - sh(a, -1, 0, 1, fill)))
        gy = (W1 * (sh(a, 0, 1, 0, fill) - sh(a, 0, -1, 0, fill))
              + W2 * (sh(a, 1, 1, 0, fill) - sh(a, -1, -1, 0, fill)
                      - sh(a, 1, -1, 0, fill) + sh(a, -1, 1, 0, fill)
                      + sh(a, 0, 1, 1, fill) - sh(a, 0, -1, -1, fill)
                      + sh(a, 0, 1, -1, fill) - sh(a, 0, -1, 1, fill)))
        gz = (W1 * (sh(a, 0, 0, 1, fill) - sh(a, 0, 0, -1, fill))
              + W2 * (sh(a, 1, 0, 1, fill) - sh(a, -1, 0, -1, fill)
                      - sh(a, 1, 0, -1, fill) + sh(a, -1, 0, 1, fill)
                      + sh(a, 0, 1, 1, fill) - sh(a, 0, -1, -1, fill)
                      - sh(a, 0, 1, -1, fill) + sh(a, 0, -1, 1, fill)))
        return gx, gy, gz

    Sw = grad(seen[0], 0.0)
    Snw = grad(seen[1], 0.0)
    A = grad(s, 1.0)
    F = []
    F.append([-G * rho[0] * Snw[a] - Ga[0] * rho[0] * A[a] for a in range(3)])
    F.append([-G * rho[1] * Sw[a] - Ga[1] * rho[1] * A[a] for a in range(3)])

    den = rho[0] / tau[0] + rho[1] / tau[1]
    den = np.where(fluid, den, 1.0)
    upx = (jx[0] / tau[0] + jx[1] / tau[1]) / den
    upy = (jy[0] / tau[0] + jy[1] / tau[1]) / den
    upz = (jz[0] / tau[0] + jz[1] / tau[1]) / den

    post = np.zeros_like(f)
    for c in (0, 1):
        r = np.where(fluid, rho[c], 1.0)
        ux = upx + tau[c] * F[c][0] / r
        uy = upy + tau[c] * F[c][1] / r
        uz = upz + tau[c] * F[c][2] / r
        uu = ux * ux + uy * uy + uz * uz
        rr = rho[c]

        def eq(wk, eu):
            return wk * rr * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu)

        feq = [eq(W0, 0.0),
               eq(W1, ux), eq(W1, -ux), eq(W1, uy), eq(W1, -uy), eq(W1, uz), eq(W1, -uz),
               eq(W2, ux + uy), eq(W2, -ux - uy), eq(W2, ux - uy), eq(W2, -ux + uy),
               eq(W2, ux + uz), eq(W2, -ux - uz), eq(W2, ux - uz), eq(W2, -ux + uz),
               eq(W2, uy + uz), eq(W2, -uy - uz), eq(W2, uy - uz), eq(W2, -uy + uz)]
        rres = res_rho(c)
        wk = [W0] + [W1] * 6 + [W2] * 12
        for k in range(19):
            v = f[c][k] - (f[c][k] - feq[k]) / tau[c]
            v = np.where(fluid, v, wk[k] * rres)
            post[c][k] = np.where(solid, 0.0, v)

    # streaming: f_k(x) <- post_k(x - e_k), or post_opp(k)(x) when x - e_k is
    # solid or beyond a wall
    def src_solid(dx, dy, dz):
        return sh(s, dx, dy, dz, 1.0) > 0.5

    new = np.zeros_like(f)
    for c in (0, 1):
        q = post[c]

        def pull(k, kop, dx, dy, dz):
            # source is x + (dx, dy, dz) = x - e_k
            b = src_solid(dx, dy, dz)
            return np.where(b, q[kop], sh(q[k], dx, dy, dz, 0.0))

        new[c][0] = q[0]
        new[c][1] = pull(1, 2, -1, 0, 0)
        new[c][2] = pull(2, 1, 1, 0, 0)
        new[c][3] = pull(3, 4, 0, -1, 0)
        new[c][4] = pull(4, 3, 0, 1, 0)
        new[c][5] = pull(5, 6, 0, 0, -1)
        new[c][6] = pull(6, 5, 0, 0, 1)
        new[c][7] = pull(7, 8, -1, -1, 0)
        new[c][8] = pull(8, 7, 1, 1, 0)
        new[c][9] = pull(9, 10, -1, 1, 0)
        new[c][10] = pull(10, 9, 1, -1, 0)
        new[c][11] = pull(11, 12, -1, 0, -1)
        new[c][12] = pull(12, 11, 1, 0, 1)
        new[c][13] = pull(13, 14, -1, 0, 1)
        new[c][14] = pull(14, 13, 1, 0, -1)
        new[c][15] = pull(15, 16, 0, -1, -1)
        new[c][16] = pull(16, 15, 0, 1, 1)
        new[c][17] = pull(17, 18, 0, -1, 1)
        new[c][18] = pull(18, 17, 0, 1, -1)
        rres = res_rho(c)
        wk = [W0] + [W1] * 6 + [W2] * 12
        for k in range(19):
            new[c][k] = np.where(fluid, new[c][k], np.where(solid, 0.0, wk[k] * rres))
    return new
