"""The kink helpers used by the full-size gradient parity test, checked with
the oracle alone: the linear-regime weights leave every unit active, a unit
planted on the kink is flagged, and flipping that unit's ReLU branch changes
the oracle gradient only inside the faces that kink_free_faces masks out."""
import numpy as np

import scenes
from oracle import adjoint as AJ
from oracle import cnn as CN
from oracle import grid as G
from tests import kinks

S, C, K = 2, 8, 3


def _case(n=32, seed=4):
    sc = scenes.plume_scene(n, seed=seed, n_obstacles=1)
    u, v = scenes.random_faces(n, n, seed, kind="mixed")
    w = scenes.random_weights(S, C, seed).astype(np.float64)
    return sc, G.plan(sc.flags), u, v, w


def test_linear_regime_keeps_every_unit_active():
    sc, P, u, v, w = _case()
    wl = kinks.linear_regime(P, u, v, sc.dx, w, S, C)
    assert np.array_equal(wl.astype(np.float32).astype(np.float64), wl)
    ratios = kinks.pre_activation_ratios(P, u, v, sc.dx, wl, S, C)
    assert min(r.min() for r in ratios) >= 1e-3
    # only the hidden biases moved
    nets0, nets1 = CN.unpack(w, S, C), CN.unpack(wl, S, C)
    for a, b in zip(nets0, nets1):
        for (W0, _), (W1, _) in zip(a["layers"], b["layers"]):
            assert np.array_equal(W0, W1)
        assert np.array_equal(a["wo"], b["wo"]) and a["bo"] == b["bo"]


def _plant(P, u, v, dx, w, k, layer, j, i, c):
    """Bias of unit (scale k, layer, channel c) that puts pixel (j, i) on the
    kink, given the forward pass below it."""
    nets = CN.unpack(w, S, C)
    d = G.divergence(P, *G.enforce_bc(P, u, v), dx)
    s = np.sqrt(np.sum(np.where(P.fluid, d, 0.0) ** 2) / P.nF)
    h = np.stack([np.where(P.fluid, d / s, 0.0), (~P.fluid).astype(np.float64)], axis=-1)
    for _ in range(k):
        h = CN.down2(h)
    for l, (W, b) in enumerate(nets[k]["layers"]):
        z = CN.conv3x3_replicate(h, W, b)
        if l == layer:
            return float(b[c] - z[j, i, c])
        h = np.maximum(z, 0.0)


def _bias_offset(k, layer):
    """Flat index of the bias of hidden layer `layer` of scale k in the
    packed parameter vector ([Cout][3][3][Cin] weights, then C biases)."""
    o = k * CN.param_count(1, C)
    for l in range(layer + 1):
        o += C * 9 * (2 if l == 0 else C)
        if l < layer:
            o += C
    return o


def test_planted_kink_is_flagged_and_stays_inside_the_mask():
    sc, P, u, v, w = _case()
    ny, nx = P.shape
    for (k, layer, j, i, c) in [(0, 1, 14, 17, 3), (1, 2, 6, 9, 5)]:
        off = _bias_offset(k, layer)
        b0 = _plant(P, u, v, sc.dx, w, k, layer, j, i, c)
        wa, wb = w.copy(), w.copy()
        # the same unit just below and just above its kink at pixel (j, i)
        A = 1e-9
        wa[off + c] = b0 - A
        wb[off + c] = b0 + A
        flagged = kinks.ambiguous_units(P, u, v, sc.dx, wa, S, C, tau=1e-6)
        assert flagged[k][j, i]
        um, vm = kinks.kink_free_faces(flagged, ny, nx)
        _, gua, gva, _ = AJ.loss_and_grad(sc.flags, u, v, sc.dx, wa, S, C, K)
        _, gub, gvb, _ = AJ.loss_and_grad(sc.flags, u, v, sc.dx, wb, S, C, K)
        du, dv = gua - gub, gva - gvb
        inside = np.sqrt(np.sum(du[~um] ** 2) + np.sum(dv[~vm] ** 2))
        assert inside > 1e-3 * np.abs(gua).max()
        # outside the mask the flip acts only through the global input scale
        # s (a multiple of d in the cell adjoint), so the difference there is
        # a multiple of D^T d (up to the forward change of the +-1e-9 bias
        # step itself, a few parts in 1e8 of the local difference)
        d = G.divergence(P, *G.enforce_bc(P, u, v), sc.dx)
        qu, qv = _dT(P, np.where(P.fluid, d, 0.0), sc.dx)
        a = (np.sum(du[um] * qu[um]) + np.sum(dv[vm] * qv[vm])) / (np.sum(qu[um] ** 2) + np.sum(qv[vm] ** 2))
        rest = np.sqrt(np.sum((du - a * qu)[um] ** 2) + np.sum((dv - a * qv)[vm] ** 2))
        assert rest <= 1e-6 * inside


def _dT(P, lam, dx):
    """Adjoint of the divergence on the planned grid: open interior and top
    faces and inflow faces (Sec. 2.1's forward difference, transposed)."""
    ny, nx = P.shape
    gu = np.zeros((ny, nx + 1))
    gv = np.zeros((ny + 1, nx))
    gu[:, 1:nx] = (lam[:, :-1] - lam[:, 1:]) / dx
    gv[1:ny] = (lam[:-1] - lam[1:]) / dx
    gv[ny] = lam[ny - 1] / dx
    gv[0] = -lam[0] / dx
    gu = np.where(P.uopen, gu, 0.0)
    gv[1:] = np.where(P.vopen[1:], gv[1:], 0.0)
    gv[0] = np.where(P.vinflow, gv[0], 0.0)
    return gu, gv
