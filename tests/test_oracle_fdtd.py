"""Pins of the oracle's Yee FDTD cavity solver.

Pins used (none re-derives the oracle's loops):
  * adjointness: the E update must apply the transpose of the H update's
    curl on the interior (PEC) E nodes -- built column by column from unit
    vectors on a 4^3 cavity;
  * discrete energy W^n = 1/2 E^n.E^n + 1/2 H^{n-1/2}.H^{n+1/2} is exactly
    conserved by the leapfrog once the source is off;
  * single cavity mode: Ez = sin(pi i/N) sin(pi j/N) (uniform in k) with H=0
    obeys e^{n+1} + e^{n-1} = (2 - dt^2 lam) e^n, lam = 8 sin^2(pi/2N), i.e.
    rotates at omega_d = (2/dt) asin((dt/2) sqrt(lam));
  * discrete Gauss law: div E changes only at the two nodes next to the
    source edge, div H stays zero;
  * PEC walls: tangential E on the walls is never changed;
  * the probe records Ez at the source after the source is added.
"""
import numpy as np
import pytest

import oracle
import synth

F = oracle.FDTD_FIELDS


def rand_fields(N, seed):
    rng = np.random.default_rng(seed)
    f = {k: rng.standard_normal((N + 1,) * 3) for k in F}
    # zero the unused padding and the PEC tangential E on the walls
    M = N + 1
    idx = np.arange(M)
    I = idx[None, None, :]
    J = idx[None, :, None]
    K = idx[:, None, None]
    inner = lambda v: (v >= 1) & (v <= N - 1)
    f["Ex"] *= (I < N) & inner(J) & inner(K)
    f["Ey"] *= (J < N) & inner(I) & inner(K)
    f["Ez"] *= (K < N) & inner(I) & inner(J)
    f["Hx"] *= (J < N) & (K < N)
    f["Hy"] *= (I < N) & (K < N)
    f["Hz"] *= (I < N) & (J < N)
    return f


def e_interior_mask(N):
    M = N + 1
    idx = np.arange(M)
    I, J, K = idx[None, None, :], idx[None, :, None], idx[:, None, None]
    inner = lambda v: (v >= 1) & (v <= N - 1)
    return {"Ex": np.broadcast_to((I < N) & inner(J) & inner(K), (M,) * 3),
            "Ey": np.broadcast_to((J < N) & inner(I) & inner(K), (M,) * 3),
            "Ez": np.broadcast_to((K < N) & inner(I) & inner(J), (M,) * 3)}


def h_mask(N):
    M = N + 1
    idx = np.arange(M)
    I, J, K = idx[None, None, :], idx[None, :, None], idx[:, None, None]
    return {"Hx": np.broadcast_to((J < N) & (K < N), (M,) * 3),
            "Hy": np.broadcast_to((I < N) & (K < N), (M,) * 3),
            "Hz": np.broadcast_to((I < N) & (J < N), (M,) * 3)}


def test_curl_adjointness_4cube():
    N, dt = 4, 0.5
    em, hm = e_interior_mask(N), h_mask(N)
    e_nodes = [(c, n) for c in ("Ex", "Ey", "Ez") for n in np.flatnonzero(em[c])]
    h_nodes = [(c, n) for c in ("Hx", "Hy", "Hz") for n in np.flatnonzero(hm[c])]
    hpos = {hn: r for r, hn in enumerate(h_nodes)}
    epos = {en: r for r, en in enumerate(e_nodes)}
    CE = np.zeros((len(h_nodes), len(e_nodes)))   # dH = -dt * CE e
    for col, (c, n) in enumerate(e_nodes):
        f = oracle.fdtd_zero_fields(N)
        f[c].flat[n] = 1.0
        g, _ = oracle.fdtd(f, N, 1, dt=dt)
        for hc in ("Hx", "Hy", "Hz"):
            for n2 in np.flatnonzero(g[hc]):
                CE[hpos[(hc, n2)], col] = -g[hc].flat[n2] / dt
    CH = np.zeros((len(e_nodes), len(h_nodes)))   # dE = dt * CH h (E starts 0)
    for col, (c, n) in enumerate(h_nodes):
        f = oracle.fdtd_zero_fields(N)
        f[c].flat[n] = 1.0
        g, _ = oracle.fdtd(f, N, 1, dt=dt)
        assert g[c].flat[n] == 1.0                 # H unchanged (E was zero)
        for ec in ("Ex", "Ey", "Ez"):
            nz = np.flatnonzero(g[ec])
            assert np.all(em[ec].flat[nz])          # only interior E changes
            for n2 in nz:
                CH[epos[(ec, n2)], col] = g[ec].flat[n2] / dt
    assert np.count_nonzero(CE) > 0
    assert np.array_equal(CH, CE.T)
    # each H face circulation has 4 edges, each interior E edge borders 4 faces
    assert set(np.unique(np.abs(CE))) <= {0.0, 1.0}


def staggered_energy(N, f0, steps, dt=0.5):
    """W^n for n = 1..steps using H at the two half steps around E^n."""
    f = f0
    out = []
    for _ in range(steps):
        hprev = {k: f[k].copy() for k in ("Hx", "Hy", "Hz")}
        f, _ = oracle.fdtd(f, N, 1, dt=dt)
        # after the step: E^{n+1}, H^{n+1/2}; energy at level n+1 needs H^{n+3/2}
        out.append((f, hprev))
    W = []
    for n in range(len(out) - 1):
        f_n, _ = out[n]
        f_next, _ = out[n + 1]
        e2 = sum(np.sum(f_n[k] ** 2) for k in ("Ex", "Ey", "Ez"))
        hh = sum(np.sum(f_n[k] * f_next[k]) for k in ("Hx", "Hy", "Hz"))
        W.append(0.5 * e2 + 0.5 * hh)
    return np.array(W)


def test_discrete_energy_conserved_float64():
    N = 6
    W = staggered_energy(N, rand_fields(N, 0), 300)
    assert np.max(np.abs(W - W[0])) / abs(W[0]) < 1e-12


def test_naive_energy_not_conserved():
    # Sanity: the collocated 1/2(E.E + H.H) oscillates, so the conservation
    # test above actually discriminates.
    N = 6
    f = rand_fields(N, 1)
    vals = []
    for _ in range(50):
        f, _ = oracle.fdtd(f, N, 1)
        vals.append(sum(np.sum(f[k] ** 2) for k in F) / 2)
    assert np.ptp(vals) / vals[0] > 1e-3


@pytest.mark.parametrize("N", [8, 16, 128])
def test_single_cavity_mode_recurrence(N):
    dt = 0.5
    M = N + 1
    i = np.arange(M)
    phi2 = np.sin(np.pi * i[None, :] / N) * np.sin(np.pi * i[:, None] / N)   # [j][i]
    f = oracle.fdtd_zero_fields(N)
    f["Ez"][:N] = phi2[None, :, :]
    steps = 40 if N == 128 else 200
    lam = 8 * np.sin(np.pi / (2 * N)) ** 2
    e = [1.0]
    g = f
    for _ in range(steps):
        g, _ = oracle.fdtd(g, N, 1, dt=dt)
        # Ez stays proportional to the mode shape
        amp = g["Ez"][N // 2, N // 2, N // 2] / phi2[N // 2, N // 2]
        assert np.max(np.abs(g["Ez"][:N] - amp * phi2[None])) < 1e-12
        e.append(amp)
    e = np.array(e)
    assert np.max(np.abs(e[2:] + e[:-2] - (2 - dt * dt * lam) * e[1:-1])) < 1e-12
    w_d = (2 / dt) * np.arcsin((dt / 2) * np.sqrt(lam))
    # closed form of the solution with H^{-1/2} = 0:  e_n = cos(n theta) + ...
    theta = w_d * dt
    alpha = (np.cos(theta) - (1 - dt * dt * lam)) / np.sin(theta)   # fixed by e_1
    ref = np.cos(theta * np.arange(steps + 1)) - alpha * np.sin(theta * np.arange(steps + 1))
    assert np.max(np.abs(e - ref)) < 1e-10
    if N == 128:
        assert abs(w_d - 0.034709587) < 5e-9


def divergence(f, kind, N):
    if kind == "E":
        X, Y, Z = f["Ex"], f["Ey"], f["Ez"]
        # node (i, j, k): (Ex[i]-Ex[i-1]) + (Ey[j]-Ey[j-1]) + (Ez[k]-Ez[k-1])
        d = (X[1:, 1:, 1:] - X[1:, 1:, :-1]) + (Y[1:, 1:, 1:] - Y[1:, :-1, 1:]) + (Z[1:, 1:, 1:] - Z[:-1, 1:, 1:])
        return d[:-1, :-1, :-1]            # interior nodes 1..N-1
    X, Y, Z = f["Hx"], f["Hy"], f["Hz"]
    # cell (i+1/2, j+1/2, k+1/2): forward differences
    return (X[:N, :N, 1:] - X[:N, :N, :-1]) + (Y[:N, 1:, :N] - Y[:N, :-1, :N]) + (Z[1:, :N, :N] - Z[:-1, :N, :N])


def test_gauss_law_and_source_location():
    N, steps = 10, 120
    src = synth.fdtd_source_cell(3, N)
    g64, _ = oracle.fdtd_pulse(steps, width=5.0, delay=20.0)
    f, probe = oracle.fdtd(oracle.fdtd_zero_fields(N), N, steps, src=src, g=g64)
    dE = divergence(f, "E", N)
    i, j, k = src
    nz = np.argwhere(np.abs(dE) > 1e-12)
    # Ez(i,j,k+1/2) feeds nodes (i,j,k) (with -) and (i,j,k+1) (with +)
    expect = {(k - 1, j - 1, i - 1), (k, j - 1, i - 1)}
    assert {tuple(v) for v in nz} <= expect
    total = np.sum(g64[:steps])
    assert abs(dE[k, j - 1, i - 1] + total) < 1e-12 * max(1, total) or k == N - 1
    assert abs(dE[k - 1, j - 1, i - 1] - total) < 1e-12 * max(1, total)
    assert np.max(np.abs(divergence(f, "H", N))) < 1e-12
    # probe = Ez at the source node after the source of that step
    assert probe[-1] == f["Ez"][k, j, i]


def test_probe_first_step_is_pulse():
    N = 8
    src = (3, 4, 2)
    g64, g32 = oracle.fdtd_pulse(4)
    _, p = oracle.fdtd(oracle.fdtd_zero_fields(N), N, 1, src=src, g=g64)
    assert p[0] == g64[0]
    _, p32 = oracle.fdtd(oracle.fdtd_zero_fields(N, np.float32), N, 1, src=src, g=g32, dtype=np.float32)
    assert p32[0] == g32[0]


def test_pulse_values():
    g64, g32 = oracle.fdtd_pulse(200, width=20.0, delay=80.0)
    assert g64[80] == 1.0
    assert abs(g64[100] - np.exp(-1.0)) < 1e-16 and abs(g64[60] - np.exp(-1.0)) < 1e-16
    assert abs(g64[0] - np.exp(-16.0)) < 1e-22
    assert np.array_equal(g32, g64.astype(np.float32))


def test_pec_tangential_e_stays_zero():
    N = 7
    f, _ = oracle.fdtd(rand_fields(N, 2), N, 30)
    em = e_interior_mask(N)
    for c in ("Ex", "Ey", "Ez"):
        assert np.all(f[c][~em[c]] == 0)


def test_float32_instantiation_matches_float64_bits_for_exact_inputs():
    # dt = 0.5 and small dyadic inputs keep every operation exact for a few
    # steps, so the two instantiations agree bit for bit.
    N = 5
    rng = np.random.default_rng(4)
    f = {k: (rng.integers(-8, 8, (N + 1,) * 3) / 8.0) for k in F}
    f = {k: v * (1.0 if k[0] == "H" else 0.0) for k, v in f.items()}
    a, _ = oracle.fdtd(f, N, 3)
    b, _ = oracle.fdtd({k: v.astype(np.float32) for k, v in f.items()}, N, 3, dtype=np.float32)
    for k in F:
        assert np.array_equal(a[k], b[k].astype(np.float64))
