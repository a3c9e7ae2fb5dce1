"""Pins of oracle.twin (the FP32 step-by-step reference) against the FP64 plain definitions."""
import math

import numpy as np
import pytest

import synth
from oracle import codec, pm, twin


@pytest.mark.parametrize("nnu", [1, 2])
def test_edge_table_is_round_to_nearest_of_eq_nu(nnu):
    m = twin.vel_m(nnu)
    g = np.random.default_rng(3)
    u = np.concatenate([g.normal(0, 1, 200000), g.standard_cauchy(50000), [0.0, -0.0, 1e30, -1e30]])
    u32 = u.astype(np.float32)
    e = twin.edge_table(nnu)
    half = (m - 1) // 2
    nu_tab = np.searchsorted(e, u32, side="right") - half
    exact = m / math.pi * np.arctan(u32.astype(np.float64))
    nu_ref = np.rint(exact)
    close = np.abs(np.abs(exact - np.floor(exact)) - 0.5) < 1e-9
    assert np.array_equal(nu_tab[~close], nu_ref[~close])
    assert nu_tab.min() >= -half and nu_tab.max() <= half


@pytest.mark.parametrize("nnu", [1, 2])
def test_decode_table_inverts_edges(nnu):
    t = twin.decode_table(nnu)
    e = twin.edge_table(nnu)
    half = (twin.vel_m(nnu) - 1) // 2
    # every table value lies inside its own bin: encode(decode(nu)) == nu for every code
    nu = np.searchsorted(e, t, side="right") - half
    assert np.array_equal(nu, np.arange(-half, half + 1))
    assert np.array_equal(t, -t[::-1])


@pytest.mark.parametrize("nchi,nnu", [(1, 1), (2, 1), (1, 2), (2, 2)])
def test_load_matches_fp64_codec(nchi, nnu):
    nc, nm = 8, 32
    x, v = synth.particle_cloud(11, 3000, nm)
    st = twin.load(x, v, nc, nchi, nnu)
    cell, chi = codec.encode_position(x / 4.0, nc, nchi)
    cid = codec.cell_id(cell, nc)
    counts, order = codec.cell_order(cid, nc**3)
    assert np.array_equal(st.cnt, counts)
    half = 1 << (8 * nchi - 1)
    assert np.array_equal(st.chi.T.astype(np.int64) - half, chi[order])
    # velocities decode to within the Eq. (v) bin of the per-cell statistics
    l, vd, cidp = twin.decode(st)
    vs = st.vs[cidp].astype(np.float64)
    u_true = (v[order].T - st.vc[:, cidp]) / vs
    u_dec = (vd - st.vc[:, cidp]) / vs
    m = twin.vel_m(nnu)
    ang = np.abs(np.arctan(u_true) - np.arctan(u_dec))
    assert ang.max() <= math.pi / (2 * m) * (1 + 1e-4) + 1e-6


@pytest.mark.parametrize("nchi", [1, 2])
def test_integer_cic_equals_fp64_cic_exactly(nchi):
    nc, nm = 8, 32
    x, v = synth.particle_cloud(12, 4000, nm)
    st = twin.load(x, v, nc, nchi, 1)
    rho = twin.deposit_int(st, nm)
    ref = pm.cic_deposit(twin.positions_fine(st), nm)
    unit = 2.0 ** (3 * (8 * nchi - 1))
    assert np.array_equal(rho.astype(np.float64) / unit, ref)
    assert rho.sum() == st.n * int(unit)


def test_move_agrees_with_fp64_formulas():
    nc, nm = 8, 32
    x, v = synth.particle_cloud(13, 5000, nm, vscale=0.5)
    st = twin.load(x, v, nc, 2, 2)
    phi = synth.smooth_potential(5, nm, amp=0.3)
    K, Dl = 0.8, 0.7
    new, info = twin.move(st, phi, np.float32(-K / 12.0), np.float32(Dl), return_info=True)
    assert not info["cfl"]
    # FP64 evaluation of the same step with the plain PM formulas of oracle.pm
    l, v32, cid = twin.decode(st)
    xpos = twin.positions_fine(st)
    grads = pm.gradient4(phi.astype(np.float64))
    acc = np.stack([-pm.cic_interp(gi, xpos) for gi in grads])
    v64 = v32.astype(np.float64) + acc * K
    x64 = np.mod(xpos.T + v64 * Dl, nm)
    assert np.allclose(info["v"], v64, rtol=0, atol=2e-6 * (1 + np.abs(v64).max()))
    # new positions decode to within half a bin (x2: 2^-15 fine cells) of the FP64 drift
    xn = twin.positions_fine(new).T
    xs = x64[:, info["perm"]]
    dx = np.abs((xn - xs + nm / 2) % nm - nm / 2)
    assert dx.max() <= 2.0**-15 + 1e-5
    assert new.cnt.sum() == st.n


def test_move_order_is_stable_within_cells():
    nc, nm = 8, 32
    x, v = synth.particle_cloud(14, 3000, nm, vscale=2.0)
    st = twin.load(x, v, nc, 1, 1)
    phi = synth.smooth_potential(6, nm)
    new, info = twin.move(st, phi, np.float32(-0.05), np.float32(0.5), return_info=True)
    perm = info["perm"]
    cnew = new.cell_of_particle()
    # inside a new cell, particles from the same source cell keep their previous order
    src = st.cell_of_particle()[perm]
    for c in np.unique(cnew)[:200]:
        sel = np.nonzero(cnew == c)[0]
        for s in np.unique(src[sel]):
            idx = perm[sel[src[sel] == s]]
            assert np.all(np.diff(idx) > 0)
    # zero drift and zero kick leaves positions and order unchanged
    same = twin.move(st, phi, np.float32(0.0), np.float32(0.0))
    assert np.array_equal(same.chi, st.chi) and np.array_equal(same.cnt, st.cnt)


def test_fma32_is_correctly_rounded():
    """fma32 against the exact rational a*b + c rounded to the nearest FP32 (ties to even)."""
    from fractions import Fraction
    g = np.random.default_rng(12)
    n = 4000
    a = g.normal(size=n).astype(np.float32) * np.float32(2.0) ** g.integers(-20, 20, n).astype(np.float32)
    b = g.normal(size=n).astype(np.float32) * np.float32(2.0) ** g.integers(-20, 20, n).astype(np.float32)
    c = g.normal(size=n).astype(np.float32) * np.float32(2.0) ** g.integers(-30, 30, n).astype(np.float32)
    c[: n // 4] = -(a[: n // 4].astype(np.float64) * b[: n // 4]).astype(np.float32)  # cancellation
    got = twin.fma32(a, b, c)

    def round_f32(x: Fraction) -> np.float32:
        f = np.float32(float(x))  # within one ulp; pick the nearest of the neighbours exactly
        cands = [np.nextafter(f, np.float32(-np.inf)), f, np.nextafter(f, np.float32(np.inf))]
        best = min(cands, key=lambda y: (abs(Fraction(float(y)) - x), int(np.float32(y).view(np.int32)) & 1))
        return best

    for i in range(n):
        exact = Fraction(float(a[i])) * Fraction(float(b[i])) + Fraction(float(c[i]))
        assert got[i] == round_f32(exact), (a[i], b[i], c[i])
    # the plain product is the special case c = 0
    assert np.array_equal(twin.fma32(a, b, np.zeros(n, np.float32)), (a * b).astype(np.float32))
