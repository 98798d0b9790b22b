"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

None of these compares the oracle with itself: each checks a closed form, an
invariant, a library routine or a brute-force/independent computation, chosen
so that a dropped term, a wrong sign or index, or a transposed operand in the
oracle fails at least one of them. Paper passages: Sec. III (lifting,
Eqs. numdens/numAtoms/Tcontribution; restricting, Eq. stress), Sec. II.B
(velocity-Verlet MD).
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle

RC = 2.5


def phi_ts(r, rc=RC):
    """LJTS pair energy written from its textbook definition (test-side)."""
    r = np.asarray(r, dtype=float)
    lj = 4.0 * (r ** -12 - r ** -6)
    return np.where(r < rc, lj - 4.0 * (rc ** -12 - rc ** -6), 0.0)


def fcc_shell_sum(rho, rc):
    """E_cold / N of the infinite FCC lattice: 1/2 sum over R != 0, |R| < rc."""
    l = (4.0 / rho) ** (1.0 / 3.0)
    m = int(math.ceil(rc / l)) + 1
    basis = np.array([[0, 0, 0], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])
    g = np.arange(-m, m + 1)
    I, J, K = np.meshgrid(g, g, g, indexing="ij")
    cells = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1).astype(float)
    R = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3) * l
    r = np.sqrt((R ** 2).sum(axis=1))
    r = r[(r > 1e-12) & (r < rc)]
    return 0.5 * phi_ts(r, rc).sum()


def two_atoms(r, L=20.0):
    x = np.array([[5.0, 5.0, 5.0], [5.0 + r, 5.0, 5.0]])
    return oracle.forces(x, L, RC)


# --- pair potential special cases (LJTS closed forms) -----------------------

def test_pair_potential_special_points():
    shift = 4.0 * (RC ** -12 - RC ** -6)
    # zero of the unshifted LJ at r = sigma
    F, U, W = two_atoms(1.0)
    assert U == pytest.approx(-shift, abs=1e-14)
    # force on atom 0 points away from atom 1 (repulsive), 24 at r = sigma
    assert F[0, 0] == pytest.approx(-24.0, rel=1e-14)
    assert F[1, 0] == pytest.approx(24.0, rel=1e-14)
    # minimum at 2^(1/6): force zero, depth -eps
    rm = 2.0 ** (1.0 / 6.0)
    F, U, W = two_atoms(rm)
    assert abs(F[0, 0]) < 1e-12
    assert U == pytest.approx(-1.0 - shift, rel=1e-13)
    # just inside the cutoff: energy continuous (-> 0), force unshifted
    F, U, W = two_atoms(RC * (1 - 1e-12))
    assert abs(U) < 1e-12
    f_rc = 24.0 * (2.0 * RC ** -13 - RC ** -7)
    assert F[1, 0] == pytest.approx(f_rc, rel=1e-9)
    # pair virial r.f
    assert W == pytest.approx(RC * f_rc, rel=1e-9)
    # at and beyond the cutoff: nothing (strict <)
    for r in (RC, RC * 1.01):
        F, U, W = two_atoms(r)
        assert U == 0.0 and W == 0.0 and not F.any()


# --- lifting geometry (Eqs. numdens, numAtoms) --------------------------------

@pytest.mark.parametrize("n_c,rho", [(2, 0.5), (3, 1.2), (4, 0.8442), (5, 0.3)])
def test_lattice_counts_and_density(n_c, rho):
    x = oracle.lattice(n_c, rho)
    N = 4 * n_c ** 3
    L = oracle.box_length(n_c, rho)
    assert x.shape == (N, 3)
    assert rho * L ** 3 == pytest.approx(N, rel=1e-14)
    assert (x >= 0).all() and (x < L).all()
    # nearest-neighbour distance of FCC is l / sqrt(2), with 12 neighbours
    l = oracle.lattice_param(rho)
    d = x[None, :, :] - x[:, None, :]
    d -= L * np.rint(d / L)
    r = np.sqrt((d ** 2).sum(-1))
    np.fill_diagonal(r, np.inf)
    assert r.min() == pytest.approx(l / math.sqrt(2), rel=1e-12)
    if n_c >= 3:
        assert ((np.abs(r - l / math.sqrt(2)) < 1e-9).sum(axis=1) == 12).all()
    # distinct sites
    assert len({tuple(np.round(p, 9)) for p in x}) == N


# --- P7: E_cold against independent shell enumeration --------------------------

@pytest.mark.parametrize("n_c,rho,rc", [(4, 0.8442, 2.5), (5, 0.3, 2.5), (5, 1.1, 2.5), (4, 1.2, 3.0), (6, 0.9, 4.0)])
def test_ecold_matches_fcc_shell_sum(n_c, rho, rc):
    N = 4 * n_c ** 3
    e_orc = oracle.ecold(n_c, rho, rc) / N
    e_ref = fcc_shell_sum(rho, rc)
    # the oracle's lattice is rounded to float (the device's storage precision);
    # forces vanish on a perfect lattice, so the rounding moves E_cold only at
    # second order in the ~1e-7 displacements: well below 1e-10 relative
    assert e_orc == pytest.approx(e_ref, rel=1e-10, abs=1e-12)


def test_ecold_is_size_independent():
    vals = [oracle.ecold(n, 0.8442, 2.5) / (4 * n ** 3) for n in (3, 4, 5, 6)]
    assert np.ptp(vals) < 1e-10


# --- P8: T = 0 virial identity W / (3V) = -dE_cold/dV -------------------------

@pytest.mark.parametrize("rho", [0.8442, 1.05, 0.62])
def test_lattice_virial_is_minus_dE_dV(rho):
    n_c, rc = 4, 2.5
    N = 4 * n_c ** 3
    x = oracle.lattice(n_c, rho)
    L = oracle.box_length(n_c, rho)
    V = L ** 3
    _, _, W = oracle.forces(x, L, rc)
    # E(V) per atom from the shell sum; rho = N / V
    h = 1e-6 * V

    def E(Vv):
        return N * fcc_shell_sum(N / Vv, rc)

    dEdV = (E(V + h) - E(V - h)) / (2 * h)
    assert W / (3 * V) == pytest.approx(-dEdV, rel=2e-6)


# --- P5: all pairs vs an independent cell list -------------------------------

@pytest.mark.parametrize("seed", [1, 2])
def test_all_pairs_equals_cell_list(seed):
    n_c, rho = 6, 0.5
    rng = np.random.default_rng(seed)
    L = oracle.box_length(n_c, rho)
    x = oracle.lattice(n_c, rho) + rng.normal(scale=0.15, size=(4 * n_c ** 3, 3))
    x -= L * np.floor(x / L)
    F1, U1, W1 = oracle.forces(x, L, RC)
    F2, U2, W2 = oracle.forces_celllist(x, L, RC)
    assert np.abs(F1 - F2).max() <= 1e-12 * np.abs(F1).max()
    assert U1 == pytest.approx(U2, rel=1e-12)
    assert W1 == pytest.approx(W2, rel=1e-12)


# --- P12: multi-image box equals its 2x2x2 replica under minimum image ----------

def test_multi_image_box_matches_replica():
    n_c, rho, rc = 3, 1.2, 3.0
    L = oracle.box_length(n_c, rho)
    assert rc > L / 2 and rc < L
    N = 4 * n_c ** 3
    assert oracle.ecold(n_c, rho, rc) / N == pytest.approx(fcc_shell_sum(rho, rc), rel=1e-10)
    rng = np.random.default_rng(3)
    x = oracle.lattice(n_c, rho) + rng.normal(scale=0.05, size=(N, 3))
    x -= L * np.floor(x / L)
    F, U, W = oracle.forces(x, L, rc)
    shifts = np.array([[a, b, c] for a in (0, 1) for b in (0, 1) for c in (0, 1)], dtype=float)
    X = (x[None, :, :] + L * shifts[:, None, :]).reshape(-1, 3)
    F8, U8, W8 = oracle.forces(X, 2 * L, rc)
    assert rc <= L  # big box uses the minimum image
    assert np.abs(F8[:N] - F).max() <= 1e-11 * np.abs(F).max()
    assert U8 == pytest.approx(8 * U, rel=1e-12)
    assert W8 == pytest.approx(8 * W, rel=1e-12)


# --- P11: Philox4x64-10 equals numpy's Philox bitwise --------------------------

@pytest.mark.parametrize("key,ctr", [((20250806, 0), (0, 0, 0, 0)), ((1, 2), (5, 0, 0, 0)),
                                     ((2 ** 64 - 1, 12345), (3 * 3999 + 2, 0, 0, 0)),
                                     ((7, 2 ** 63), (2 ** 40, 3, 9, 1))])
def test_philox_matches_numpy(key, ctr):
    mine = oracle.philox4x64_10(key, ctr)
    # numpy's Philox increments its 256-bit counter before each block
    c = list(ctr)
    for i in range(4):
        if c[i] > 0:
            c[i] -= 1
            break
        c[i] = 2 ** 64 - 1
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(c, dtype=np.uint64))
    ref = np.array([bg.random_raw() for _ in range(4)], dtype=np.uint64)
    assert (mine == ref).all()


def test_gaussian_draws_are_standard_normal():
    z = np.array([oracle.gauss(99, 3, a, c) for a in range(4000) for c in range(3)])
    assert abs(z.mean()) < 4 / math.sqrt(z.size)
    assert abs(z.var() - 1) < 4 * math.sqrt(2 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-3


def test_gaussian_box_muller_definition():
    # first two Philox words -> Box-Muller, written out here from the textbook form
    w = oracle.philox4x64_10((11, 4), (3 * 17 + 1, 0, 0, 0))
    u1 = 1.0 - float(int(w[0]) >> 11) * 2.0 ** -53
    u2 = float(int(w[1]) >> 11) * 2.0 ** -53
    z = math.sqrt(-2 * math.log(u1)) * math.cos(2 * math.pi * u2)
    assert oracle.gauss(11, 4, 17, 1) == pytest.approx(z, rel=1e-15, abs=1e-15)


# --- P9: lifting invariants ---------------------------------------------------

@pytest.mark.parametrize("n_c,rho,T", [(4, 0.8442, 0.722), (2, 0.3, 2.0), (5, 1.1, 3.0)])
def test_lift_invariants(n_c, rho, T):
    N = 4 * n_c ** 3
    e = 1.5 * T * (1 - 1 / N)
    cell = oracle.Cell(rho=rho, e=e, n_c=n_c, seed=5, cell_id=9)
    x, v, Ec = oracle.lift(cell)
    assert np.array_equal(x, x.astype(np.float32).astype(np.float64))
    assert np.array_equal(v, v.astype(np.float32).astype(np.float64))
    K = 0.5 * (v ** 2).sum()
    assert K == pytest.approx(N * e, rel=1e-6)  # exact in FP64 before rounding to float
    assert np.abs(v.sum(axis=0)).max() < 1e-5 * np.abs(v).sum()
    # first-guess temperature 2E/N_DOF equals T when e = N_DOF T / (2N)
    assert 2 * N * e / (3 * N - 3) == pytest.approx(T, rel=1e-14)
    assert Ec == pytest.approx(oracle.ecold(n_c, rho, 2.5), rel=1e-15)


def test_rescale_pins_energy_above_cold():
    cell = oracle.Cell(rho=0.8442, e=1.0788, n_c=4, dt=0.005)
    sch = oracle.Schedule(n_steps=300, n_avg=100, rescale_steps=(50, 150))
    r = oracle.run(cell, sch)
    for k in (50, 150):
        assert (r.K[k] + r.U[k] - r.Ecold_total) / cell.N == pytest.approx(cell.e, rel=1e-12)
    # between re-pins the energy is conserved (NVE), so the pin only corrects
    # the small integration error
    E = r.K + r.U - r.Ecold_total
    assert np.abs(E[51:150] / cell.N - cell.e).max() < 1e-3


def test_below_cold_flag():
    # a target energy below the cold lattice after a disordering run: start hot,
    # then demand e = 0 at a re-pin once E_pot > E_cold
    cell = oracle.Cell(rho=0.8442, e=2.0, n_c=3, dt=0.005)
    x, v, Ec = oracle.lift(cell)
    cold = oracle.Cell(rho=0.8442, e=1e-9, n_c=3, dt=0.005)
    r = oracle.run(cold, oracle.Schedule(n_steps=100, n_avg=50, rescale_steps=(60,)), x=x, v=v, Ecold_total=Ec)
    assert r.result.status & oracle.BELOW_COLD


# --- P1 / P2: Newton's third law and momentum ----------------------------------

def test_newton3_and_momentum():
    cell = oracle.Cell(rho=0.9, e=1.5, n_c=3, dt=0.005, seed=3)
    x, v, Ec = oracle.lift(cell)
    v = v - v.mean(axis=0)
    r = oracle.run(cell, oracle.Schedule(n_steps=200, n_avg=100), x=x, v=v, Ecold_total=Ec, n_recF=50)
    for k in range(50):
        F = r.F[k]
        # step 0 is the lattice, where every force nearly cancels: the floor
        # 1e-14 N covers the rounding of the O(10) pair forces themselves
        assert np.abs(F.sum(axis=0)).max() <= 1e-12 * np.abs(F).sum() + 1e-14 * cell.N
    assert np.abs(r.v.sum(axis=0)).max() <= 1e-12 * np.abs(r.v).sum()


# --- P4: time reversibility ------------------------------------------------------

def test_time_reversibility():
    cell = oracle.Cell(rho=0.8, e=1.2, n_c=3, dt=0.004, seed=8)
    x0, v0, Ec = oracle.lift(cell)
    sch = oracle.Schedule(n_steps=20, n_avg=10, n_blocks=2)
    a = oracle.run(cell, sch, x=x0, v=v0, Ecold_total=Ec)
    b = oracle.run(cell, sch, x=a.x, v=-a.v, Ecold_total=Ec)
    L = oracle.box_length(cell.n_c, cell.rho)
    d = b.x - x0
    d -= L * np.rint(d / L)
    assert np.abs(d).max() <= 1e-9
    assert np.abs(b.v + v0).max() <= 1e-9


# --- P3: velocity-Verlet energy error scales as dt^2 -------------------------------

def test_nve_energy_error_scales_as_dt_squared():
    cell = oracle.Cell(rho=0.8442, e=1.5, n_c=3, dt=0.004, seed=2)
    x, v, Ec = oracle.lift(cell)
    eq = oracle.run(cell, oracle.Schedule(n_steps=400, n_avg=100), x=x, v=v, Ecold_total=Ec)
    fl = []
    for dt, n in ((0.004, 200), (0.002, 400)):
        c = oracle.Cell(rho=cell.rho, e=cell.e, n_c=cell.n_c, dt=dt)
        r = oracle.run(c, oracle.Schedule(n_steps=n, n_avg=n // 2), x=eq.x, v=eq.v, Ecold_total=Ec)
        E = r.K + r.U
        fl.append(np.sqrt(np.mean((E - E.mean()) ** 2)))
    ratio = fl[0] / fl[1]
    assert 3.0 < ratio < 5.0, ratio


# --- P6: ideal-gas limits -------------------------------------------------------

def test_ideal_gas_without_potential():
    cell = oracle.Cell(rho=0.5, e=1.3, n_c=3, dt=0.005, seed=4)
    N = cell.N
    sch = oracle.Schedule(n_steps=200, n_avg=100, eps=0.0)
    r = oracle.run(cell, sch)
    L = oracle.box_length(cell.n_c, cell.rho)
    V = L ** 3
    np.testing.assert_allclose(r.P, 2 * r.K / (3 * V), rtol=1e-14)
    np.testing.assert_allclose(r.P, cell.rho * r.T * (1 - 1 / N), rtol=1e-13)
    assert r.result.P == pytest.approx(cell.rho * r.result.T * (1 - 1 / N), rel=1e-13)
    assert r.result.P_se < 1e-12


def b2_ljts(T, rc=RC):
    """Second virial coefficient of the LJTS fluid by 1-D quadrature (SciPy)."""
    f = lambda r: (math.exp(-float(phi_ts(r, rc)) / T) - 1.0) * r * r
    pts = [0.8, 1.0, 2 ** (1 / 6), 1.5]
    val, _ = integrate.quad(f, 1e-6, rc, points=pts, limit=400)
    return -2 * math.pi * val


def test_low_density_virial_limit():
    rho, T = 0.02, 2.0
    n_c = 4
    N = 4 * n_c ** 3
    e = 1.5 * T * (1 - 1 / N)
    Z = []
    for s in range(6):
        cell = oracle.Cell(rho=rho, e=e, n_c=n_c, dt=0.005, seed=100 + s)
        sch = oracle.Schedule(n_steps=4000, n_avg=3000, rescale_steps=(300, 700))
        r = oracle.run(cell, sch)
        Tm = r.result.T
        Z.append(r.result.P / (rho * Tm) - (1 - 1 / N))
        T_used = Tm
    Z = np.array(Z)
    se = Z.std(ddof=1) / math.sqrt(len(Z))
    b2 = b2_ljts(T_used)
    # third virial term bounded by rho^2 (|B3| < 1 at these T)
    assert abs(Z.mean() - b2 * rho) <= 3 * se + rho ** 2, (Z.mean(), b2 * rho, se)
    assert b2 < 0  # attractive regime at T = 2


# --- P10: block standard error on an AR(1) series --------------------------------

def test_block_se_matches_ar1_analytic():
    from scipy.signal import lfilter

    rng = np.random.default_rng(11)
    phi, n, B, reps = 0.9, 20_000, 10, 400
    sig = math.sqrt(1 - phi ** 2)
    se2, means = [], []
    for _ in range(reps):
        # stationary unit-variance AR(1): x_t = phi x_{t-1} + sqrt(1 - phi^2) eps_t
        x0 = rng.normal()
        x = lfilter([sig], [1.0, -phi], rng.normal(size=n), zi=[phi * x0])[0]
        m, se = oracle.block_stats(x, B)
        assert m == pytest.approx(x.mean(), rel=1e-12, abs=1e-15)
        se2.append(se * se)
        means.append(m)
    analytic2 = (1 + phi) / ((1 - phi) * n)
    # SE^2 of B blocks is an unbiased estimate of the variance of the mean; its
    # average over the replicas has relative sampling error sqrt(2/(B-1)/reps)
    tol = 3.5 * math.sqrt(2 / (B - 1) / reps)
    assert np.mean(se2) == pytest.approx(analytic2, rel=tol)
    # and the observed spread of the means agrees too
    assert np.var(means, ddof=1) == pytest.approx(analytic2, rel=3.5 * math.sqrt(2 / reps))


# --- thermostatted lifting and canonical production (GJF Langevin) -----------

def test_thermostat_noise_definition():
    # one Philox block at counter (atom, step, 1, query), numpy's generator
    # for the words, Box-Muller written out here: (cos, sin) of words 0-1,
    # cos of 2-3
    key, a, k, q = (11, 4), 17, 9, 3
    c = [a - 1, k, 1, q]  # numpy pre-increments the counter
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(c, dtype=np.uint64))
    w = [int(bg.random_raw()) for _ in range(4)]
    u = [1.0 - (w[0] >> 11) * 2.0 ** -53, (w[1] >> 11) * 2.0 ** -53,
         1.0 - (w[2] >> 11) * 2.0 ** -53, (w[3] >> 11) * 2.0 ** -53]
    r1, r2 = math.sqrt(-2 * math.log(u[0])), math.sqrt(-2 * math.log(u[2]))
    want = [r1 * math.cos(2 * math.pi * u[1]), r1 * math.sin(2 * math.pi * u[1]), r2 * math.cos(2 * math.pi * u[3])]
    assert oracle.noise3(*key, a, k, q) == pytest.approx(want, rel=1e-14, abs=1e-15)
    assert np.abs(oracle.noise3(*key, a, k, 0) - oracle.noise3(*key, a, k, q)).max() > 0.01
    z = np.array([oracle.noise3(5, 2, a, k) for a in range(300) for k in range(1, 8)]).ravel()
    assert abs(z.mean()) < 4 / math.sqrt(z.size) and abs(z.var() - 1) < 4 * math.sqrt(2 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-3


def test_gjf_without_friction_is_velocity_verlet():
    """gamma = 0 makes a = b = 1 and the noise zero: the GJF step is then the
    velocity-Verlet step (rearranged, so equal up to rounding)."""
    cell = oracle.Cell(rho=0.8, e=1.5, n_c=3, rc=2.5, dt=0.005, seed=3, cell_id=1)
    x0, v0, Ec = oracle.lift(cell)
    a = oracle.run(cell, oracle.Schedule(200, 100, n_blocks=10), x=x0, v=v0, Ecold_total=Ec)
    b = oracle.run(cell, oracle.Schedule(200, 100, n_blocks=10, ensemble=1, gamma=0.0), x=x0, v=v0, Ecold_total=Ec)
    assert np.abs(a.x - b.x).max() < 1e-9 and np.abs(a.v - b.v).max() < 1e-9
    assert np.abs(a.U - b.U).max() < 1e-9 * abs(a.U).max()


@pytest.mark.parametrize("gamma,dt", [(5.0, 0.02), (0.5, 0.005)])
def test_gjf_free_particles_sample_the_exact_temperature(gamma, dt):
    """With the potential off, GJF's on-site velocities have stationary
    variance exactly T per component for any dt: v' = a v + b beta gives
    <v^2> = b^2 2 gamma T dt / (1 - a^2) = T. A wrong damping or noise factor
    shows up at order gamma dt (10 % for the first case)."""
    N = 256
    T = 1.7
    cell = oracle.Cell(rho=0.5, e=1.5 * T * (1 - 1 / N), n_c=4, rc=2.5, dt=dt, seed=21, cell_id=5)
    r = oracle.run(cell, oracle.Schedule(6000, 5000, n_blocks=20, ensemble=1, gamma=gamma, eps=0.0))
    t = 2 * r.K[1001:] / (3 * N)  # per-component variance of the velocities
    m, se = oracle.block_stats(t, 20)
    assert abs(m - T) <= 4 * se and abs(m - T) <= 0.02 * T, (m, se)


# --- full stress tensor (Eq. stress) ----------------------------------------

def _cluster():
    """A compact 38-atom FCC fragment in the middle of a large box (no image
    within rc), slightly perturbed so that no symmetry hides a component."""
    L = 40.0
    x = oracle.lattice(3, 1.0)
    c = x.mean(0)
    x = x[np.linalg.norm(x - c, axis=1) < 2.6]
    x = x + np.random.default_rng(4).normal(scale=0.05, size=x.shape) + (L / 2 - c)
    return x, L


@pytest.mark.parametrize("a,b", [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)])
def test_virial_tensor_is_minus_the_strain_derivative(a, b):
    """For an isolated cluster and the affine map x_a -> x_a + e x_b,
    dE/de = sum over pairs phi'(r) d_a d_b / r = -sum d_a f_b: the virial
    tensor component (a, b) is minus the strain derivative of E_pot. Central
    differences of E_pot (the pinned scalar path) fix each component's index
    mapping and sign."""
    x, L = _cluster()
    rc = 2.5
    comp = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (0, 1): 3, (0, 2): 4, (1, 2): 5}[(a, b)]
    S = oracle.virial_tensor(x, L, rc)
    h = 1e-6
    E = []
    for e in (h, -h):
        y = x.copy()
        y[:, a] += e * (x[:, b] - L / 2)
        E.append(oracle.forces(y, L, rc)[1])
    dE = (E[0] - E[1]) / (2 * h)
    assert S[comp] == pytest.approx(-dE, rel=1e-6, abs=1e-7)


def test_virial_tensor_trace_is_the_scalar_virial():
    cell = oracle.Cell(rho=0.9, e=2.0, n_c=3, rc=2.5, dt=0.004, seed=1, cell_id=2)
    r = oracle.run(cell, oracle.Schedule(50, 10, n_blocks=2))
    L = oracle.box_length(3, 0.9)
    S = oracle.virial_tensor(r.x, L, 2.5)
    W = oracle.forces(r.x, L, 2.5)[2]
    assert S[0] + S[1] + S[2] == pytest.approx(W, rel=1e-12)


def test_stress_of_an_equilibrium_liquid_is_isotropic():
    """<sigma> of a liquid: equal diagonal, vanishing shear, trace/3 = <P>
    (on the sampled steps, within the statistical error of the averages)."""
    cell = oracle.Cell(rho=0.7, e=float(1.5 * 2.0 * (1 - 1 / 256)), n_c=4, rc=2.5, dt=0.005, seed=9, cell_id=0)
    r = oracle.run(cell, oracle.Schedule(3000, 2500, rescale_steps=(250, 500), energy_every=1))
    s = np.array(r.result.stress)
    P = r.result.P
    se = 4 * max(r.result.P_se, 1e-3)
    assert np.all(np.abs(s[:3] - P) < 3 * se), (s, P, se)
    assert np.all(np.abs(s[3:]) < 3 * se), (s, se)
    assert s[:3].mean() == pytest.approx(P, abs=1e-9)  # every window step sampled: trace/3 is P exactly


# --- embedded-atom form (Eq. Etot): Sutton-Chen (9, 6) stand-in, shifted force --

EAM_C, EAM_RC = 39.432, 1.5


def _sf(g, dg, r, rc):
    """Shifted-force truncation written from its definition (test side)."""
    r = np.asarray(r, dtype=float)
    return np.where(r < rc, g(r) - g(rc) - (r - rc) * dg(rc), 0.0)


def eam_V(r, rc):
    return _sf(lambda s: s ** -9.0, lambda s: -9.0 * s ** -10.0, r, rc)


def eam_f(r, rc):
    return _sf(lambda s: s ** -6.0, lambda s: -6.0 * s ** -7.0, r, rc)


def fcc_distances(rho, rc):
    """|R| of every FCC lattice vector R != 0 with |R| < rc."""
    l = (4.0 / rho) ** (1.0 / 3.0)
    m = int(math.ceil(rc / l)) + 1
    basis = np.array([[0, 0, 0], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])
    g = np.arange(-m, m + 1)
    I, J, K = np.meshgrid(g, g, g, indexing="ij")
    cells = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1).astype(float)
    R = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3) * l
    r = np.sqrt((R ** 2).sum(axis=1))
    return r[(r > 1e-12) & (r < rc)]


def eam_lattice_energy(rho, rc, c=EAM_C):
    """E/N of the perfect FCC lattice: every site sees the same density, so
    E/N = 1/2 sum_R V(|R|) + F(sum_R f(|R|)) with F = -c sqrt."""
    r = fcc_distances(rho, rc)
    return 0.5 * eam_V(r, rc).sum() - c * math.sqrt(eam_f(r, rc).sum())


def _eam_cell(rho, n_c, rc=EAM_RC, **kw):
    return oracle.Cell(rho=rho, e=kw.pop("e", 20.0), n_c=n_c, rc=rc, dt=kw.pop("dt", 0.001), potential=1,
                       eam_c=EAM_C, **kw)


def _eam_disordered(n_c=3, rho=4.2, amp=0.06, seed=0):
    rng = np.random.default_rng(seed)
    x = oracle.lattice(n_c, rho) + rng.uniform(-amp, amp, size=(4 * n_c ** 3, 3))
    return x, oracle.box_length(n_c, rho)


@pytest.mark.parametrize("n_c,rho,rc", [(3, 4.0, 1.5), (4, 4.6, 1.5), (3, 3.4, 1.45), (4, 5.5, 1.8), (2, 4.0, 1.2)])
def test_eam_ecold_matches_the_lattice_sum(n_c, rho, rc):
    cell = _eam_cell(rho, n_c, rc)
    assert oracle.ecold_cell(cell) / cell.N == pytest.approx(eam_lattice_energy(rho, rc), rel=1e-10)


@pytest.mark.parametrize("rho", [3.6, 4.0, 5.0])
def test_eam_lattice_virial_is_minus_dE_dV(rho):
    """The T = 0 virial identity W / (3V) = -dE/dV holds for the many-body
    energy too (it depends on interatomic distances only)."""
    n_c, rc = 3, EAM_RC
    N = 4 * n_c ** 3
    x = oracle.lattice(n_c, rho)
    L = oracle.box_length(n_c, rho)
    V = L ** 3
    W = oracle.forces_eam(x, L, rc, EAM_C)[2]
    h = 1e-6 * V
    dEdV = N * (eam_lattice_energy(N / (V + h), rc) - eam_lattice_energy(N / (V - h), rc)) / (2 * h)
    assert W / (3 * V) == pytest.approx(-dEdV, rel=2e-6)


@pytest.mark.parametrize("n_c,rho,rc", [(3, 4.2, 1.5), (2, 4.2, 1.5)], ids=["minimum-image", "multi-image"])
def test_eam_forces_are_minus_the_energy_gradient(n_c, rho, rc):
    """Central differences of E_pot: a dropped embedding term (F'_i or F'_j),
    a wrong sign or a wrong derivative of V or f fails this."""
    x, L = _eam_disordered(n_c, rho)
    F, U, W, S, rb = oracle.forces_eam(x, L, rc, EAM_C)
    rng = np.random.default_rng(1)
    h = 1e-5
    scale = np.abs(F).max()
    for _ in range(12):
        i, a = int(rng.integers(len(x))), int(rng.integers(3))
        E = []
        for s in (h, -h):
            y = x.copy()
            y[i, a] += s
            E.append(oracle.forces_eam(y, L, rc, EAM_C)[1])
        assert F[i, a] == pytest.approx(-(E[0] - E[1]) / (2 * h), abs=2e-6 * scale)


def test_eam_dimer_closed_form():
    """Two atoms: E = V_s(r) + 2 F(f_s(r)); the force is -dE/dr along the bond."""
    rc = EAM_RC
    for r in (0.65, 0.8, 1.1, 1.45):
        x = np.array([[5.0, 5.0, 5.0], [5.0 + r, 5.0, 5.0]])
        F, U, W, S, rb = oracle.forces_eam(x, 20.0, rc, EAM_C)
        f = float(eam_f(r, rc))
        assert rb == pytest.approx([f, f], rel=1e-13)
        assert U == pytest.approx(float(eam_V(r, rc)) - 2 * EAM_C * math.sqrt(f), rel=1e-13)
        dV = -9.0 * (r ** -10 - rc ** -10)
        df = -6.0 * (r ** -7 - rc ** -7)
        dE = dV + 2 * (-EAM_C / (2 * math.sqrt(f))) * df
        assert F[1, 0] == pytest.approx(-dE, rel=1e-12) and F[0, 0] == pytest.approx(dE, rel=1e-12)
        assert W == pytest.approx(-dE * r, rel=1e-12)


def test_eam_newton3_and_momentum():
    x, L = _eam_disordered(3, 4.5, seed=3)
    F = oracle.forces_eam(x, L, EAM_RC, EAM_C)[0]
    assert np.abs(F.sum(axis=0)).max() < 1e-9 * np.abs(F).max()


@pytest.mark.parametrize("a,b", [(0, 0), (1, 2), (2, 0)])
def test_eam_virial_tensor_is_minus_the_strain_derivative(a, b):
    """Isolated cluster, affine map x_a -> x_a + e x_b: dE/de = -S_ab."""
    rng = np.random.default_rng(5)
    x = oracle.lattice(2, 4.0) + rng.uniform(-0.05, 0.05, size=(32, 3)) + 9.0
    L = 20.0
    comp = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (0, 1): 3, (0, 2): 4, (1, 2): 5}[tuple(sorted((a, b)))]
    S = oracle.forces_eam(x, L, EAM_RC, EAM_C)[3]
    h = 1e-6
    E = []
    for e in (h, -h):
        y = x.copy()
        y[:, a] += e * (x[:, b] - L / 2)
        E.append(oracle.forces_eam(y, L, EAM_RC, EAM_C)[1])
    assert S[comp] == pytest.approx(-(E[0] - E[1]) / (2 * h), rel=1e-6, abs=1e-6)


def test_eam_nve_energy_error_scales_as_dt_squared():
    cell = _eam_cell(4.0, 3, e=20.0, seed=2)
    x, v, Ec = oracle.lift(cell)
    fl = []
    for dt, n in ((0.002, 200), (0.001, 400)):
        c = _eam_cell(4.0, 3, e=20.0, seed=2, dt=dt)
        r = oracle.run(c, oracle.Schedule(n_steps=n, n_avg=n // 2), x=x, v=v, Ecold_total=Ec)
        E = r.K + r.U
        fl.append(np.sqrt(np.mean((E - E.mean()) ** 2)))
    assert 3.0 < fl[0] / fl[1] < 5.0, fl


def test_eam_lift_pins_the_energy_above_cold():
    """The lifting operator is potential-agnostic: K = N e on the lattice."""
    cell = _eam_cell(4.4, 3, e=15.0, seed=4)
    x, v, Ec = oracle.lift(cell)
    assert Ec == pytest.approx(oracle.ecold_cell(cell), rel=1e-15)
    assert 0.5 * (v ** 2).sum() == pytest.approx(cell.N * cell.e, rel=1e-6)
