"""Pins of the FP64 CPU oracle against facts the paper and the mathematics fix.

None of these tests compares the oracle with itself: each checks it against a
textbook constant, a closed form, an invariant, a finite-difference gradient,
a brute-force definition or the statistics the paper states (Sec. 2.1).
"""
import math
import os

import numpy as np
import pytest

import gen
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden(name):
    with open(os.path.join(HERE, "golden", name)) as f:
        vals = [line for line in f if line.strip() and not line.startswith("#")]
    return float(vals[0])


def nacl(cells=2):
    """Rock-salt crystal with nearest-neighbour distance 1 (2*cells per axis)."""
    g = np.arange(2 * cells, dtype=np.float64)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    x, y, z = (a.ravel().copy() for a in (X, Y, Z))
    q = (-1.0) ** (x + y + z)
    return x, y, z, q, float(2 * cells)


def random_ions(n, L, seed, dmin=0.8):
    x, y, z = gen.rsa_positions(seed, 0, n, [L, L, L], dmin)
    q = gen.charges(seed, 0, n, n // 2, n // 2)
    return x, y, z, q


# --------------------------------------------------------------------------
# Exact Ewald sum (Eq. 3-6): Madelung constant, alpha independence, gradients
# --------------------------------------------------------------------------
@pytest.mark.parametrize("alpha", [1.0, 1.5])
def test_nacl_madelung(alpha):
    x, y, z, q, L = nacl()
    r = oracle.ewald_exact(x, y, z, q, L, alpha)
    M = _golden("nacl_madelung.txt")
    assert abs(-2.0 * r["u"] / len(x) - M) < 1e-10
    # every ion of a perfect crystal is a centre of inversion symmetry
    assert np.abs(r["F"]).max() < 1e-12


def test_ewald_alpha_independence():
    x, y, z, q = random_ions(8, 5.0, 11)
    r1 = oracle.ewald_exact(x, y, z, q, 5.0, 0.8)
    r2 = oracle.ewald_exact(x, y, z, q, 5.0, 2.0)
    assert abs(r1["u"] - r2["u"]) < 1e-11 * abs(r1["u"])
    assert np.abs(r1["F"] - r2["F"]).max() < 1e-11 * np.abs(r1["F"]).max()
    # and the split parts differ, so the check is not vacuous
    assert abs(r1["u_real"] - r2["u_real"]) > 1e-3


def test_ewald_force_is_minus_gradient():
    x, y, z, q = random_ions(8, 5.0, 12)
    L, a, h = 5.0, 1.2, 1e-5
    F = oracle.ewald_exact(x, y, z, q, L, a)["F"]
    coords = [x, y, z]
    for i in (0, 3, 6):
        for d in range(3):
            cp = [c.copy() for c in coords]
            cm = [c.copy() for c in coords]
            cp[d][i] += h
            cm[d][i] -= h
            up = oracle.ewald_exact(*cp, q, L, a)["u"]
            um = oracle.ewald_exact(*cm, q, L, a)["u"]
            fd = -(up - um) / (2 * h)
            assert abs(fd - F[i, d]) < 1e-6 * max(1.0, abs(F[i, d]))


# --------------------------------------------------------------------------
# Fourier part for a fixed mode set (Eq. 5, 7, 9)
# --------------------------------------------------------------------------
def _random_modes(P, mmax, seed):
    rng = np.random.default_rng(seed)
    m = rng.integers(-mmax, mmax + 1, size=(3, P)).astype(np.int32)
    m[:, np.all(m == 0, axis=0)] = 1
    w = rng.uniform(0.1, 1.0, P)
    return m, w


def test_fourier_zero_net_force_any_modes():
    x, y, z, q = random_ions(200, 9.0, 13)
    m, w = _random_modes(64, 6, 1)
    F, _, _ = oracle.fourier_force(x, y, z, q, 9.0, m, w)
    assert np.abs(F.sum(axis=0)).max() < 1e-12 * np.abs(F).sum()


def test_fourier_zero_on_perfect_crystal():
    x, y, z, q, L = nacl()
    m, w = _random_modes(128, 8, 2)
    F, re, im = oracle.fourier_force(x, y, z, q, L, m, w)
    assert np.abs(F).max() < 1e-11
    # the structure factor is real and equals N on the crystal's reciprocal lattice, 0 elsewhere
    on = np.all(np.mod(m, 4) == 2, axis=0)
    assert np.allclose(re[on], len(x), atol=1e-10) and np.allclose(re[~on], 0.0, atol=1e-10)
    assert np.abs(im).max() < 1e-10


def test_fourier_force_is_minus_gradient_of_fixed_mode_energy():
    x, y, z, q = random_ions(12, 6.0, 14)
    L, h = 6.0, 1e-6
    m, w = _random_modes(40, 5, 3)
    F, _, _ = oracle.fourier_force(x, y, z, q, L, m, w)
    coords = [x, y, z]
    for i in (0, 5, 11):
        for d in range(3):
            cp = [c.copy() for c in coords]
            cm = [c.copy() for c in coords]
            cp[d][i] += h
            cm[d][i] -= h
            up = oracle.fourier_energy(w, *oracle.rho(*cp, q, L, m))
            um = oracle.fourier_energy(w, *oracle.rho(*cm, q, L, m))
            fd = -(up - um) / (2 * h)
            assert abs(fd - F[i, d]) < 1e-6 * max(1.0, np.abs(F[i]).max())


def test_fourier_mode_sign_symmetry_and_translation():
    x, y, z, q = random_ions(50, 7.0, 15)
    m, w = _random_modes(30, 5, 4)
    F1, _, _ = oracle.fourier_force(x, y, z, q, 7.0, m, w)
    F2, _, _ = oracle.fourier_force(x, y, z, q, 7.0, -m, w)  # k and -k give the same term
    assert np.abs(F1 - F2).max() < 1e-12 * np.abs(F1).max()
    F3, _, _ = oracle.fourier_force(x + 1.3, y - 2.1, z + 0.4, q, 7.0, m, w)
    assert np.abs(F1 - F3).max() < 1e-11 * np.abs(F1).max()


def test_full_lattice_reproduces_ewald_reciprocal():
    """Deterministic full-lattice weights 4 pi e^{-k^2/4a}/(V k^2): the fixed-mode
    energy is the exact U^F of Eq. 5, and near + Fourier forces are the exact
    Ewald force (alpha large enough that the minimum image holds the real part)."""
    x, y, z, q = random_ions(8, 6.0, 16)
    L, a = 6.0, 4.0
    ex = oracle.ewald_exact(x, y, z, q, L, a)
    M = oracle.axis_cutoff(L, a) + 1
    m, w = oracle.full_lattice(L, a, [M, M, M])
    re, im = oracle.rho(x, y, z, q, L, m)
    assert abs(oracle.fourier_energy(w, re, im) - ex["u_recip"]) < 1e-12 * abs(ex["u_recip"])
    F, _, _ = oracle.fourier_force(x, y, z, q, L, m, w, re, im)
    s = oracle.make_sys(L, a, r_coul=L / 2, r_lj=0.0)
    FN = oracle.real_force(x, y, z, q, np.arange(8, dtype=np.int32), s, oracle.COUL_REAL)
    assert np.abs(F + FN - ex["F"]).max() < 1e-12 * np.abs(ex["F"]).max()


# --------------------------------------------------------------------------
# Importance sampling of the modes (Eq. 9): distribution, normalizer, bias
# --------------------------------------------------------------------------
def test_normalizer_closed_form_vs_direct_sum():
    for L, a in [(6.0, 0.3), (9.0, 1.0), (30.0, 0.3)]:
        M = oracle.axis_cutoff(L, a)
        g = np.arange(-M, M + 1)
        k2 = (2 * np.pi * g / L) ** 2
        K2 = k2[:, None, None] + k2[None, :, None] + k2[None, None, :]
        direct = np.exp(-K2 / (4 * a)).sum() - 1.0
        S = oracle.norm_S(L, a)
        assert abs(S - direct) < 1e-12 * direct
        # Poisson summation: H = L sqrt(a/pi) up to exponentially small terms for large L
        if L * math.sqrt(a) > 10:
            assert abs(oracle.axis_H(L, a) - L * math.sqrt(a / math.pi)) < 1e-10


def test_sampler_marginal_chi2():
    from scipy import stats
    L, a, P = 8.0, 0.6, 512
    draws = np.concatenate([oracle.sample_k(7, e, L, a, P)[0] for e in range(40)], axis=1)
    assert not np.any(np.all(draws == 0, axis=0))
    M = oracle.axis_cutoff(L, a)
    g = np.arange(-M, M + 1)
    pm = np.exp(-(np.pi * g / L) ** 2 / a)
    H = pm.sum()
    # marginal of one axis given m != 0: p(m) (H^2 - [m == 0]) / (H^3 - 1)
    for d in range(3):
        expect = pm * (H * H - (g == 0)) / (H ** 3 - 1)
        counts = np.array([(draws[d] == v).sum() for v in g])
        keep = expect * draws.shape[1] > 5
        e = expect[keep] * draws.shape[1]
        obs = counts[keep]
        e = e * obs.sum() / e.sum()
        chi2 = ((obs - e) ** 2 / e).sum()
        pval = stats.chi2.sf(chi2, keep.sum() - 1)
        assert pval > 1e-3, (d, chi2, pval)


def test_sampler_weights_and_determinism():
    L, a, P = 10.0, 0.5, 64
    m1, w1 = oracle.sample_k(3, 5, L, a, P)
    m2, w2 = oracle.sample_k(3, 5, L, a, P)
    assert np.array_equal(m1, m2) and np.array_equal(w1, w2)
    m3, _ = oracle.sample_k(3, 6, L, a, P)
    assert not np.array_equal(m1, m3)
    k2 = ((2 * np.pi * m1 / L) ** 2).sum(axis=0)
    S = oracle.norm_S(L, a)
    assert np.allclose(w1, S / P * 4 * np.pi / (L ** 3 * k2), rtol=1e-14)


@pytest.mark.slow
def test_rbe_unbiased_mean_converges_to_ewald():
    """The mean of the Eq. 9 estimate over independent mode draws converges
    to the exact Fourier force of Eq. 7, with error falling like M^{-1/2}."""
    x, y, z, q = random_ions(8, 5.0, 17)
    L, a, P = 5.0, 1.0, 8
    M = oracle.axis_cutoff(L, a) + 1
    mf, wf = oracle.full_lattice(L, a, [M, M, M])
    Fex, _, _ = oracle.fourier_force(x, y, z, q, L, mf, wf)
    acc = np.zeros_like(Fex)
    errs = {}
    for e in range(1, 16385):
        m, w = oracle.sample_k(99, e, L, a, P)
        acc += oracle.fourier_force(x, y, z, q, L, m, w)[0]
        if e in (256, 1024, 4096, 16384):
            errs[e] = np.linalg.norm(acc / e - Fex) / np.linalg.norm(Fex)
    assert errs[16384] < 0.03
    assert errs[16384] < errs[256] / 3.0


# --------------------------------------------------------------------------
# Real space (Eq. 2, 7, 8) and the random batch list (Eq. 10-12)
# --------------------------------------------------------------------------
def _lj_ions(n, L, seed, frac=0.5):
    x, y, z = gen.rsa_positions(seed, 0, n, [L, L, L], 0.8)
    nq = int(round(n * frac / 2))
    q = gen.charges(seed, 0, n, nq, nq)
    return x, y, z, q, np.arange(n, dtype=np.int32)


def test_real_space_cells_match_brute_force():
    x, y, z, q, ids = _lj_ions(3000, 16.0, 21)
    s = oracle.make_sys(16.0, 0.35, 5.0, 2.5)
    Fb = oracle.real_force(x, y, z, q, ids, s)
    Fc = oracle.real_force(x, y, z, q, ids, s, cells=True)
    assert np.abs(Fb - Fc).max() < 1e-12 * np.abs(Fb).max()
    # Newton's third law: without the random batch list the pair sum cancels
    assert np.abs(Fb.sum(axis=0)).max() < 1e-10 * np.abs(Fb).sum() / len(x)


def test_real_space_force_is_minus_gradient():
    x, y, z, q, ids = _lj_ions(60, 6.0, 22)
    s = oracle.make_sys(6.0, 0.5, 2.9, 2.5)
    F = oracle.real_force(x, y, z, q, ids, s)
    h = 1e-6
    coords = [x, y, z]
    for i in (0, 17, 42):
        for d in range(3):
            cp = [c.copy() for c in coords]
            cm = [c.copy() for c in coords]
            cp[d][i] += h
            cm[d][i] -= h
            up = sum(oracle.real_energy(*cp, q, s))
            um = sum(oracle.real_energy(*cm, q, s))
            fd = -(up - um) / (2 * h)
            assert abs(fd - F[i, d]) < 1e-5 * max(1.0, np.abs(F[i]).max())


def test_real_space_single_pair_closed_form():
    """Two opposite charges at distance r along x: Eq. 8 by hand."""
    r, a = 1.3, 0.4
    x = np.array([0.0, r]); y = np.zeros(2); z = np.zeros(2); q = np.array([1.0, -1.0])
    s = oracle.make_sys(20.0, a, 5.0, 2.5)
    F = oracle.real_force(x, y, z, q, np.arange(2, dtype=np.int32), s)
    sa = math.sqrt(a)
    G = math.erfc(sa * r) / r ** 3 + 2 * sa * math.exp(-a * r * r) / (math.sqrt(math.pi) * r * r)
    GLJ = 24 * (2 / r ** 14 - 1 / r ** 8)
    fx0 = (-1.0 * G + GLJ) * (0.0 - r)  # on particle 0, d = r_0 - r_1 = -r
    assert abs(F[0, 0] - fx0) < 1e-14 * abs(fx0)
    assert abs(F[1, 0] + fx0) < 1e-14 * abs(fx0)


def test_rbl_reduces_to_full_cutoff_when_batch_covers_shell():
    x, y, z, q, ids = _lj_ions(2000, 14.0, 23, frac=0.25)
    full = oracle.make_sys(14.0, 0.35, 6.0, 2.5)
    rbl = oracle.make_sys(14.0, 0.35, 6.0, 2.5, r_core=3.0, p_shell=100000)
    Ff = oracle.real_force(x, y, z, q, ids, full)
    Fr, nsh = oracle.real_force(x, y, z, q, ids, rbl, seed=5, ev=1, return_nshell=True)
    assert np.abs(Ff - Fr).max() < 1e-12 * np.abs(Ff).max()
    charged = q != 0
    assert np.all(nsh[charged] > 100) and np.all(nsh[~charged] == -1)


def test_rbl_shell_counts_and_batch():
    x, y, z, q, ids = _lj_ions(1500, 12.0, 24, frac=0.25)
    rbl = oracle.make_sys(12.0, 0.35, 6.0, 2.5, r_core=3.0, p_shell=20)
    _, nsh = oracle.real_force(x, y, z, q, ids, rbl, seed=5, ev=1, return_nshell=True)
    # brute-force shell size for a few charged particles (all species in the shell)
    for i in np.flatnonzero(q != 0)[:5]:
        d = np.stack([x - x[i], y - y[i], z - z[i]], axis=1)
        d -= 12.0 * np.rint(d / 12.0)
        r2 = (d ** 2).sum(axis=1)
        r2[i] = -1
        assert nsh[i] == np.count_nonzero((r2 > 9.0) & (r2 <= 36.0))


def test_rbl_unbiased_over_seeds():
    """Mean over independent batches of the Eq. 11 estimate -> full-cutoff force."""
    x, y, z, q, ids = _lj_ions(800, 11.0, 25, frac=0.5)
    full = oracle.make_sys(11.0, 0.35, 5.4, 2.5)
    rbl = oracle.make_sys(11.0, 0.35, 5.4, 2.5, r_core=2.7, p_shell=10)
    idx = np.flatnonzero(q != 0)[:40]
    Ff = oracle.real_force(x, y, z, q, ids, full, idx=idx)
    acc = np.zeros_like(Ff)
    errs = {}
    for e in range(1, 1025):
        acc += oracle.real_force(x, y, z, q, ids, rbl, seed=77, ev=e, idx=idx)
        if e in (64, 1024):
            errs[e] = np.linalg.norm(acc / e - Ff) / np.linalg.norm(Ff)
    assert errs[1024] < errs[64] / 2.5
    assert errs[1024] < 0.02


def test_rbl_momentum_correction():
    x, y, z, q, ids = _lj_ions(1500, 12.0, 26, frac=0.25)
    rbl = oracle.make_sys(12.0, 0.35, 6.0, 2.5, r_core=3.0, p_shell=20)
    F = oracle.real_force(x, y, z, q, ids, rbl, seed=8, ev=2)
    assert np.abs(F.sum(axis=0)).max() > 1e-6  # the raw estimate does not conserve momentum
    Fc, mean = oracle.mean_correct(F)
    assert np.abs(Fc.sum(axis=0)).max() < 1e-9
    assert np.allclose(mean, F.mean(axis=0), rtol=1e-12, atol=0)


def test_rbl_key_is_bijection_in_j():
    keys = {oracle.rbl_key(1, 2, 3, j) for j in range(20000)}
    assert len(keys) == 20000


# --------------------------------------------------------------------------
# Binning: stable counting sort by (species, cell)
# --------------------------------------------------------------------------
def test_binning_against_brute_force():
    n, L = 5000, 17.0
    x, y, z, q, _ = _lj_ions(n, L, 31, frac=0.3)
    x = x.copy(); x[:5] = [0.0, L - 1e-13, -1e-18, L, 2 * L + 0.5]  # edge values
    nc = np.array([6, 5, 7], np.int32)
    cs, perm = oracle.bin_cells(x, y, z, q, L, nc)
    assert np.array_equal(np.sort(perm), np.arange(n))
    # brute-force key in numpy
    def wrap(v):
        w = v - L * np.floor(v / L)
        w[(w < 0) | (w >= L)] = 0.0
        return w
    c = [np.minimum((wrap(v) * (nc[d] / L)).astype(np.int64), nc[d] - 1) for d, v in enumerate((x, y, z))]
    ncell = int(np.prod(nc))
    key = np.where(q == 0, ncell, 0) + (c[2] * nc[1] + c[1]) * nc[0] + c[0]
    ref = np.argsort(key, kind="stable")
    assert np.array_equal(perm, ref)
    counts = np.bincount(key, minlength=2 * ncell)
    assert np.array_equal(np.diff(cs), counts) and cs[0] == 0 and cs[-1] == n


# --------------------------------------------------------------------------
# Velocity Verlet
# --------------------------------------------------------------------------
def test_free_flight_is_exact():
    n, L = 100, 10.0
    x, y, z = gen.rsa_positions(41, 0, n, [L] * 3, 0.8)
    v = np.stack(gen.velocities(41, 0, n), axis=1)
    r = np.stack([x, y, z], axis=1)
    for _ in range(10):
        r = oracle.drift_wrap(r, v, 0.01, L)
    ref = np.stack([x, y, z], axis=1) + 0.1 * v  # 10 drifts of 0.01
    ref = ref - L * np.floor(ref / L)
    d = (r - ref + L / 2) % L - L / 2
    assert np.abs(d).max() < 1e-12


def _vv(r, v, q, L, s, m, w, dt, steps):
    ids = np.arange(len(q), dtype=np.int32)
    def force(r):
        return oracle.total_force(r[:, 0], r[:, 1], r[:, 2], q, ids, s, m, w)["F"]
    F = force(r)
    for _ in range(steps):
        v = oracle.kick(F, v, dt / 2)
        r = oracle.drift_wrap(r, v, dt, L)
        F = force(r)
        v = oracle.kick(F, v, dt / 2)
    return r, v


def test_vv_time_reversible_with_fixed_modes():
    n, L = 40, 8.0
    x, y, z, q = random_ions(n, L, 42)
    s = oracle.make_sys(L, 0.6, 3.9, 2.5)
    m, w = oracle.sample_k(1, 0, L, 0.6, 20)
    r0 = np.stack([x, y, z], axis=1)
    v0 = np.stack(gen.velocities(42, 0, n), axis=1)
    r1, v1 = _vv(r0, v0, q, L, s, m, w, 0.002, 25)
    r2, v2 = _vv(r1, -v1, q, L, s, m, w, 0.002, 25)
    d = (r2 - r0 + L / 2) % L - L / 2
    assert np.abs(d).max() < 1e-9
    assert np.abs(v2 + v0).max() < 1e-8


@pytest.mark.slow
def test_vv_energy_error_scales_as_dt_squared():
    """With the exact Ewald force the energy error of velocity Verlet is O(dt^2)."""
    n, L, a = 8, 5.0, 1.0
    x, y, z, q = random_ions(n, L, 43)
    r0 = np.stack([x, y, z], axis=1)
    v0 = 0.5 * np.stack(gen.velocities(43, 0, n), axis=1)

    def energy_dev(dt, T=0.2):
        r, v = r0.copy(), v0.copy()
        ex = oracle.ewald_exact(r[:, 0], r[:, 1], r[:, 2], q, L, a)
        e0 = ex["u"] + 0.5 * (v ** 2).sum()
        F = ex["F"]
        dev = 0.0
        for _ in range(int(round(T / dt))):
            v = v + 0.5 * dt * F
            r = oracle.drift_wrap(r, v, dt, L)
            ex = oracle.ewald_exact(r[:, 0], r[:, 1], r[:, 2], q, L, a, tol=1e-14)
            F = ex["F"]
            v = v + 0.5 * dt * F
            dev = max(dev, abs(ex["u"] + 0.5 * (v ** 2).sum() - e0))
        return dev

    d1, d2 = energy_dev(0.02), energy_dev(0.01)
    assert 2.5 < d1 / d2 < 6.0, (d1, d2)


def test_total_force_is_minus_gradient_of_energy_terms_with_prefactor():
    """With a Coulomb prefactor kc != 1 and a fixed mode sample, the total
    force without the random batch list (Eq. 7-9) is minus the gradient of
    coul_real + lj + fourier - self: kc must scale the real-space, Fourier
    and self terms alike (the self term is constant in the positions)."""
    x, y, z, q, ids = _lj_ions(40, 6.0, 31)
    kc = 2.5
    s = oracle.make_sys(6.0, 0.5, 2.9, 2.5, kc=kc)
    m, w = _random_modes(24, 4, 9)
    F = oracle.total_force(x, y, z, q, ids, s, m, w, components=False)["F"]
    h = 1e-6
    coords = [x, y, z]
    for i in (0, 11, 33):
        for d in range(3):
            cp = [c.copy() for c in coords]
            cm = [c.copy() for c in coords]
            cp[d][i] += h
            cm[d][i] -= h
            up = oracle.energy_terms(*cp, q, s, m, w)["potential"]
            um = oracle.energy_terms(*cm, q, s, m, w)["potential"]
            fd = -(up - um) / (2 * h)
            assert abs(fd - F[i, d]) < 1e-5 * max(1.0, np.abs(F[i]).max())
    # the prefactor is linear in every Coulomb term
    e1 = oracle.energy_terms(x, y, z, q, oracle.make_sys(6.0, 0.5, 2.9, 2.5), m, w)
    e2 = oracle.energy_terms(x, y, z, q, s, m, w)
    for k in ("coul_real", "fourier", "self"):
        assert e2[k] == pytest.approx(kc * e1[k], rel=1e-14)
    assert e2["lj"] == e1["lj"]


def test_self_and_kinetic_energy_closed_forms():
    """Eq. 6 for a +-q pair is 2 q^2 sqrt(a/pi); (m/2)|v|^2 for one particle."""
    a = 0.37
    assert oracle.self_energy(np.array([1.5, -1.5]), a) == pytest.approx(2 * 2.25 * math.sqrt(a / math.pi),
                                                                         rel=1e-15)
    assert oracle.kinetic_energy(np.array([[1.0, 2.0, -2.0]]), 3.0) == pytest.approx(13.5, rel=1e-15)


def _dilated_real_energy(x, y, z, q, L, s, alpha, r_coul, r_lj):
    sys_s = oracle.make_sys(L * s, alpha, r_coul, r_lj)
    return sum(oracle.real_energy(x * s, y * s, z * s, q, sys_s))


def test_real_virial_is_minus_dilation_derivative():
    """W = sum d.F = -dU/ds for positions and box scaled by s (cutoffs fixed;
    no pair sits within the step of a cutoff)."""
    x, y, z, q, ids = _lj_ions(60, 7.0, 41)
    sys = oracle.make_sys(7.0, 0.5, 3.2, 2.5)
    wc, wl = oracle.real_virial(x, y, z, q, sys)
    h = 1e-7
    up = _dilated_real_energy(x, y, z, q, 7.0, 1 + h, 0.5, 3.2, 2.5)
    um = _dilated_real_energy(x, y, z, q, 7.0, 1 - h, 0.5, 3.2, 2.5)
    fd = -(up - um) / (2 * h)
    assert fd == pytest.approx(wc + wl, rel=1e-6, abs=1e-6)


def test_fourier_virial_is_minus_dilation_derivative_of_exact_reciprocal_energy():
    """With the deterministic full-lattice weights 4 pi exp(-k^2/4a)/(V k^2)
    the fixed-mode energy is the exact reciprocal energy of Eq. 5; its
    dilation derivative (weights recomputed at the scaled box, rho unchanged)
    is minus the virial formula."""
    x, y, z, q = random_ions(30, 6.0, 42)
    alpha, L, mmax = 0.6, 6.0, (6, 6, 6)
    m, w = oracle.full_lattice(L, alpha, mmax)
    re, im = oracle.rho(x, y, z, q, L, m)
    W = oracle.fourier_virial(m, L, alpha, w, re, im)
    h = 1e-6
    u = []
    for s in (1 + h, 1 - h):
        _, ws = oracle.full_lattice(L * s, alpha, mmax)
        u.append(oracle.fourier_energy(ws, re, im))  # rho is dilation invariant (k.r fixed)
    fd = -(u[0] - u[1]) / (2 * h)
    assert fd == pytest.approx(W, rel=1e-7)


def test_coulomb_virial_theorem_for_the_full_ewald_sum():
    """The Ewald energy of a neutral periodic system is homogeneous of degree
    -1 under dilation, so the Coulomb virial equals the total Coulomb energy:
    W_real + W_recip = U_real + U_recip - U_self (real space converged inside
    L/2, reciprocal sum over the full lattice)."""
    x, y, z, q = random_ions(40, 10.0, 43)
    L, alpha, rc = 10.0, 1.39, 5.0  # erfc(sqrt(a) rc) ~ 1e-16
    sys = oracle.make_sys(L, alpha, rc, 2.5)
    uc, _ = oracle.real_energy(x, y, z, q, sys)
    wc, _ = oracle.real_virial(x, y, z, q, sys)
    m, w = oracle.full_lattice(L, alpha, (24, 24, 24))
    re, im = oracle.rho(x, y, z, q, L, m)
    uk = oracle.fourier_energy(w, re, im)
    wk = oracle.fourier_virial(m, L, alpha, w, re, im)
    us = oracle.self_energy(q, alpha)
    ex = oracle.ewald_exact(x, y, z, q, L, alpha)
    assert uc + uk - us == pytest.approx(ex["u"], rel=1e-12)
    assert wc + wk == pytest.approx(uc + uk - us, rel=1e-11)


def _nvt(r, v, xi, eta, q, L, s, m, w, dt, steps, kT, tau):
    ids = np.arange(len(q), dtype=np.int32)

    def force(r):
        return oracle.total_force(r[:, 0], r[:, 1], r[:, 2], q, ids, s, m, w)["F"]
    F = force(r)
    for _ in range(steps):
        r, v, F, xi, eta = oracle.nvt_step(r, v, F, xi, eta, force, dt, L, 1.0, kT, tau)
    return r, v, xi, eta


def test_nvt_time_reversible_with_fixed_modes():
    """The Nose-Hoover equations are reversible under (v, xi) -> (-v, -xi);
    the symmetric split keeps that exactly, up to rounding."""
    n, L = 40, 8.0
    x, y, z, q = random_ions(n, L, 44)
    s = oracle.make_sys(L, 0.6, 3.9, 2.5)
    m, w = oracle.sample_k(1, 0, L, 0.6, 20)
    r0 = np.stack([x, y, z], axis=1)
    v0 = np.stack(gen.velocities(44, 0, n), axis=1)
    r1, v1, xi1, eta1 = _nvt(r0, v0, 0.3, 0.0, q, L, s, m, w, 0.002, 25, 0.5, 0.05)
    assert abs(xi1 - 0.3) > 1e-3  # the thermostat did act
    r2, v2, xi2, eta2 = _nvt(r1, -v1, -xi1, eta1, q, L, s, m, w, 0.002, 25, 0.5, 0.05)
    d = (r2 - r0 + L / 2) % L - L / 2
    assert np.abs(d).max() < 1e-9
    assert np.abs(v2 + v0).max() < 1e-8
    assert abs(xi2 + 0.3) < 1e-9 and abs(eta2) < 1e-9


def test_nvt_with_infinite_thermostat_mass_is_nve():
    """Q -> infinity leaves xi at 0, so every scaling is exactly 1."""
    n, L = 40, 8.0
    x, y, z, q = random_ions(n, L, 45)
    s = oracle.make_sys(L, 0.6, 3.9, 2.5)
    m, w = oracle.sample_k(1, 0, L, 0.6, 20)
    r0 = np.stack([x, y, z], axis=1)
    v0 = np.stack(gen.velocities(45, 0, n), axis=1)
    r1, v1 = _vv(r0, v0, q, L, s, m, w, 0.002, 10)
    r2, v2, xi, _ = _nvt(r0, v0, 0.0, 0.0, q, L, s, m, w, 0.002, 10, 0.5, 1e12)
    assert np.array_equal(r1, r2) and np.array_equal(v1, v2) and abs(xi) < 1e-20


@pytest.mark.slow
def test_nvt_conserved_quantity_error_scales_as_dt_squared():
    """With the exact Ewald force, K + U + Q xi^2/2 + N_f kT eta is conserved
    by the Nose-Hoover dynamics; the integrator's error in it is O(dt^2)."""
    n, L, a, kT, tau = 8, 5.0, 1.0, 0.5, 0.05
    x, y, z, q = random_ions(n, L, 46)
    r0 = np.stack([x, y, z], axis=1)
    v0 = 0.5 * np.stack(gen.velocities(46, 0, n), axis=1)
    nf = 3.0 * n - 3.0
    Q = nf * kT * tau * tau

    def force(r):
        return oracle.ewald_exact(r[:, 0], r[:, 1], r[:, 2], q, L, a, tol=1e-14)

    def h_dev(dt, T=0.2):
        r, v, xi, eta = r0.copy(), v0.copy(), 0.0, 0.0
        ex = force(r)
        F = ex["F"]
        h0 = ex["u"] + oracle.kinetic_energy(v, 1.0)
        dev, last = 0.0, {}

        def fwrap(rr):
            last["ex"] = force(rr)
            return last["ex"]["F"]
        for _ in range(int(round(T / dt))):
            r, v, F, xi, eta = oracle.nvt_step(r, v, F, xi, eta, fwrap, dt, L, 1.0, kT, tau)
            h = last["ex"]["u"] + oracle.kinetic_energy(v, 1.0) + 0.5 * Q * xi * xi + nf * kT * eta
            dev = max(dev, abs(h - h0))
        return dev, xi

    (d1, xi1), (d2, _) = h_dev(0.02), h_dev(0.01)
    assert abs(xi1) > 1e-2  # the thermostat is active over the run
    assert 2.5 < d1 / d2 < 6.0, (d1, d2)


# --------------------------------------------------------------------------
# Alternative proposal P(k) ~ exp(-k^2/4a)/k^2 (kdist = 1)
# --------------------------------------------------------------------------
def test_norm_S2_equals_its_integral_representation():
    """1/k^2 = int_0^inf exp(-t k^2) dt turns S2 into a 1-D integral of products
    of 1-D lattice sums over the same truncated lattice (an independent way
    to the same number)."""
    from scipy.integrate import quad
    L, a = (5.0, 6.0, 7.5), 1.1
    Ms = [oracle.axis_cutoff(Ld, a) for Ld in L]

    def integrand(t):
        prod = 1.0
        for Ld, M in zip(L, Ms):
            k = 2 * math.pi * np.arange(-M, M + 1) / Ld
            prod *= np.exp(-(1.0 / (4 * a) + t) * k * k).sum()
        return prod - 1.0
    val, err = quad(integrand, 0.0, np.inf, epsabs=0.0, epsrel=1e-12, limit=400)
    assert oracle.norm_S2(L, a) == pytest.approx(val, rel=1e-9)


def test_over_k2_sample_frequencies():
    """Draw frequencies of the most likely modes match
    exp(-k^2/4a)/(k^2 S2) within 4 standard errors."""
    L, a, P = 6.0, 0.8, 4000
    S2 = oracle.norm_S2(L, a)
    counts = {}
    ndraw = 0
    for e in range(10):
        m, w = oracle.sample_k(5, e, L, a, P, kdist=1)
        assert np.allclose(w, S2 / P * 4 * math.pi / L ** 3, rtol=1e-15)
        for c in map(tuple, m.T):
            counts[c] = counts.get(c, 0) + 1
        ndraw += P
    for mv in [(1, 0, 0), (0, -1, 0), (0, 0, 1), (1, 1, 0), (-1, 0, 1), (1, 1, 1)]:
        k2 = sum((2 * math.pi * c / L) ** 2 for c in mv)
        p = math.exp(-k2 / (4 * a)) / k2 / S2
        se = math.sqrt(p * (1 - p) / ndraw)
        assert abs(counts.get(mv, 0) / ndraw - p) < 4 * se, mv


def test_over_k2_estimator_unbiased():
    """The mean of the Fourier estimate with the exp(-k^2/4a)/k^2 proposal and
    its weights (S2/P) 4 pi / V converges to the exact Fourier force."""
    x, y, z, q = random_ions(8, 5.0, 17)
    L, a, P = 5.0, 1.0, 8
    M = oracle.axis_cutoff(L, a) + 1
    mf, wf = oracle.full_lattice(L, a, [M, M, M])
    Fex, _, _ = oracle.fourier_force(x, y, z, q, L, mf, wf)
    acc = np.zeros_like(Fex)
    errs = {}
    for e in range(1, 8193):
        m, w = oracle.sample_k(98, e, L, a, P, kdist=1)
        acc += oracle.fourier_force(x, y, z, q, L, m, w)[0]
        if e in (128, 8192):
            errs[e] = np.linalg.norm(acc / e - Fex) / np.linalg.norm(Fex)
    assert errs[8192] < 0.04
    assert errs[8192] < errs[128] / 3.0


# --------------------------------------------------------------------------
# Variant: shell of charged particles only (r_lj <= r_core)
# --------------------------------------------------------------------------
def test_charged_shell_counts_and_full_cutoff_limit():
    """The charged-only shell holds exactly the charged j in (r_core, r_coul];
    with a batch covering it the estimate is the full-cutoff force (the
    neutral j it leaves out carry no force beyond the core)."""
    x, y, z, q, ids = _lj_ions(1500, 12.0, 27, frac=0.25)
    full = oracle.make_sys(12.0, 0.35, 6.0, 2.5)
    chg = oracle.make_sys(12.0, 0.35, 6.0, 2.5, r_core=3.0, p_shell=100000, shell_charged=1)
    Fr, nsh = oracle.real_force(x, y, z, q, ids, chg, seed=5, ev=1, return_nshell=True)
    Ff = oracle.real_force(x, y, z, q, ids, full)
    assert np.abs(Ff - Fr).max() < 1e-12 * np.abs(Ff).max()
    for i in np.flatnonzero(q != 0)[:5]:
        d = np.stack([x - x[i], y - y[i], z - z[i]], axis=1)
        d -= 12.0 * np.rint(d / 12.0)
        r2 = (d ** 2).sum(axis=1)
        r2[i] = -1
        assert nsh[i] == np.count_nonzero((r2 > 9.0) & (r2 <= 36.0) & (q != 0))
    assert np.all(nsh[q == 0] == -1)


def test_charged_shell_unbiased_over_seeds():
    x, y, z, q, ids = _lj_ions(800, 11.0, 28, frac=0.5)
    full = oracle.make_sys(11.0, 0.35, 5.4, 2.5)
    chg = oracle.make_sys(11.0, 0.35, 5.4, 2.5, r_core=2.7, p_shell=10, shell_charged=1)
    idx = np.flatnonzero(q != 0)[:40]
    Ff = oracle.real_force(x, y, z, q, ids, full, idx=idx)
    acc = np.zeros_like(Ff)
    errs = {}
    for e in range(1, 1025):
        acc += oracle.real_force(x, y, z, q, ids, chg, seed=78, ev=e, idx=idx)
        if e in (64, 1024):
            errs[e] = np.linalg.norm(acc / e - Ff) / np.linalg.norm(Ff)
    assert errs[1024] < errs[64] / 2.5
    assert errs[1024] < 0.02


def test_splitmix64_matches_the_published_sequence():
    """The oracle's stream output n = mix64(seed + (n + 1) gamma) reproduces
    SplitMix64's reference outputs from state 0, so the draws of Eq. 9 and
    the keys of Eq. 11 come from the published generator."""
    with open(os.path.join(HERE, "golden", "splitmix64_seed0.txt")) as f:
        ref = [int(line, 16) for line in f if line.strip() and not line.startswith("#")]
    gamma = 0x9E3779B97F4A7C15
    got = [oracle.mix64(((n + 1) * gamma) & (2 ** 64 - 1)) for n in range(len(ref))]
    assert got == ref
