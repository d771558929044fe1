"""Pins of the CPU oracle against mathematics it does not itself use.

The paper prints no worked numerical example for the Poisson solve, so every
pin here comes from a definition, a closed form, an invariant or a library
routine:

* the recursive mixed-radix FFT against the direct DFT sum and numpy's FFT;
* plane waves, whose potential is known in closed form (Eq. (6) for a single
  Fourier component), in cubic, orthorhombic and triclinic cells;
* Poisson's equation itself, checked with numpy's own transforms;
* invariants of the Poisson operator: symmetry, positivity, null space,
  scaling with the cell, translation;
* the Hartree energy of periodic Gaussians from a direct reciprocal-space sum
  and, for one Gaussian, from the Ewald closed form;
* Hartree forces from the analytic reciprocal-space derivative and from
  finite differences;
* the splat against a brute-force per-point image sum.
"""
import numpy as np
import pytest
from scipy.special import erfc

from paper_1209_4506_amd import inputs

# Madelung constant of the simple-cubic lattice of unit charges in a uniform
# neutralizing background (energy per charge -alpha/(2L) for edge L).
MADELUNG_SC = 2.8372974794806


def recip_np(cell):
    """Reciprocal rows via numpy's matrix inverse: B = 2 pi inv(A)^T."""
    return 2.0 * np.pi * np.linalg.inv(np.asarray(cell, float)).T


def grid_points(cell, dims):
    i, j, k = np.meshgrid(*[np.arange(n) / n for n in dims], indexing="ij")
    frac = np.stack([i, j, k], -1)
    return frac @ np.asarray(cell, float)


def smooth_sizes(limit, primes=(2, 3, 5)):
    out = []
    for n in range(1, limit + 1):
        m = n
        for p in primes:
            while m % p == 0:
                m //= p
        if m == 1:
            out.append(n)
    return out


# --------------------------------------------------------------------- FFT


@pytest.mark.parametrize("n", smooth_sizes(16) + [7, 11, 13, 14, 21, 49])
def test_fft1d_vs_direct_dft(oracle_mod, n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    t = np.arange(n)
    W = np.exp(-2j * np.pi * np.outer(t, t) / n)
    ref = W @ x
    got = oracle_mod.fft1d(x, -1)
    assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))
    back = oracle_mod.fft1d(x, +1)
    refb = np.conj(W) @ x
    assert np.max(np.abs(back - refb)) <= 1e-13 * max(1.0, np.max(np.abs(refb)))


def test_fft3d_vs_direct_dft_tiny(oracle_mod):
    """Every 2/3/5-smooth size up to 16 appears on some axis of a tiny 3-D grid."""
    sizes = smooth_sizes(16)
    rng = np.random.default_rng(5)
    for t in range(len(sizes)):
        dims = (sizes[t], sizes[(t + 3) % len(sizes)], sizes[(t + 7) % len(sizes)])
        x = rng.standard_normal(dims) + 1j * rng.standard_normal(dims)
        ref = x.astype(complex)
        for ax, n in enumerate(dims):
            tt = np.arange(n)
            W = np.exp(-2j * np.pi * np.outer(tt, tt) / n)
            ref = np.moveaxis(np.tensordot(W, np.moveaxis(ref, ax, 0), axes=(1, 0)), 0, ax)
        got = oracle_mod.fft3d(x, -1)
        assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref)), dims


@pytest.mark.parametrize("dims", [(24, 30, 32), (45, 36, 40), (9, 50, 27)])
def test_fft3d_vs_numpy(oracle_mod, dims):
    rng = np.random.default_rng(sum(dims))
    x = rng.standard_normal(dims) + 1j * rng.standard_normal(dims)
    ref = np.fft.fftn(x)
    assert np.max(np.abs(oracle_mod.fft3d(x, -1) - ref)) <= 1e-13 * np.max(np.abs(ref))
    refi = np.fft.ifftn(x) * x.size
    assert np.max(np.abs(oracle_mod.fft3d(x, +1) - refi)) <= 1e-13 * np.max(np.abs(refi))


# ------------------------------------------------------ Poisson: plane waves

CELLS = {
    "cubic": np.diag([10.0, 10.0, 10.0]),
    "ortho": np.diag([8.0, 11.0, 13.5]),
    "triclinic": np.array([[9.0, 0.0, 0.0], [2.5, 8.0, 0.0], [-1.5, 2.0, 10.5]]),
}


@pytest.mark.parametrize("cellname", list(CELLS))
@pytest.mark.parametrize("m0", [(1, 0, 0), (2, -3, 1), (0, 4, -5), (3, 3, 3)])
@pytest.mark.parametrize("wave", ["cos", "sin"])
def test_plane_wave(oracle_mod, cellname, m0, wave):
    cell = CELLS[cellname]
    dims = (16, 18, 15)
    G0 = np.asarray(m0, float) @ recip_np(cell)
    r = grid_points(cell, dims)
    phase = r @ G0
    rho = np.cos(phase) if wave == "cos" else np.sin(phase)
    V, e_real, e_recip, mi = oracle_mod.poisson(cell.reshape(9), rho)
    g2 = float(G0 @ G0)
    omega = abs(np.linalg.det(cell))
    assert np.max(np.abs(V - 4 * np.pi / g2 * rho)) <= 1e-13 * 4 * np.pi / g2
    assert abs(e_real - np.pi * omega / g2) <= 1e-13 * np.pi * omega / g2
    assert abs(e_recip - e_real) <= 1e-13 * abs(e_real)
    assert mi <= 1e-13 * np.max(np.abs(V))


@pytest.mark.parametrize("cellname", ["cubic", "ortho"])
def test_plane_wave_nyquist(oracle_mod, cellname):
    """A wave at the Nyquist index of one even axis is +-1 on the grid."""
    cell = CELLS[cellname]
    dims = (16, 12, 10)
    G0 = np.array([8.0, 0.0, 0.0]) @ recip_np(cell)
    rho = np.cos(grid_points(cell, dims) @ G0)
    V, e_real, e_recip, _ = oracle_mod.poisson(cell.reshape(9), rho)
    g2 = float(G0 @ G0)
    omega = abs(np.linalg.det(cell))
    assert np.max(np.abs(V - 4 * np.pi / g2 * rho)) <= 1e-13 * 4 * np.pi / g2
    assert abs(e_real - 2 * np.pi * omega / g2) <= 1e-13 * 2 * np.pi * omega / g2
    assert abs(e_recip - e_real) <= 1e-13 * e_real


def test_energy_sums_on_a_large_grid(oracle_mod):
    """Both E_H forms of a plane wave on 192^3 points (7.1M terms) against
    the closed form pi Omega / |G0|^2 at 1e-14: a plain running sum of that
    many terms loses about 1e-11 to rounding, the compensated sums keep the
    value to a few ulps."""
    cell = CELLS["triclinic"] * 1.5
    dims = (192, 192, 192)
    G0 = np.array([5.0, -7.0, 11.0]) @ recip_np(cell)
    rho = np.cos(grid_points(cell, dims) @ G0)
    V, e_real, e_recip, _ = oracle_mod.poisson(cell.reshape(9), rho)
    e_cf = np.pi * abs(np.linalg.det(cell)) / float(G0 @ G0)
    assert abs(e_real - e_cf) <= 1e-14 * e_cf
    assert abs(e_recip - e_cf) <= 1e-14 * e_cf


# ------------------------------------------- Poisson's equation, by numpy


@pytest.mark.parametrize("cellname", list(CELLS))
def test_poisson_equation_spectral(oracle_mod, cellname):
    """-Laplacian(V) = 4 pi (rho - mean rho), the Laplacian taken with numpy's
    FFT and numpy's reciprocal basis.  Odd dims avoid any Nyquist ambiguity."""
    cell = CELLS[cellname]
    dims = (15, 21, 25)
    rho = inputs.random_grid(dims, 11)
    V, _, _, _ = oracle_mod.poisson(cell.reshape(9), rho)
    B = recip_np(cell)
    m = [np.fft.fftfreq(n, 1.0 / n) for n in dims]
    M = np.stack(np.meshgrid(*m, indexing="ij"), -1)
    G = M @ B
    g2 = np.sum(G * G, -1)
    lap = np.real(np.fft.ifftn(g2 * np.fft.fftn(V)))
    assert np.max(np.abs(lap - 4 * np.pi * (rho - rho.mean()))) <= 1e-11 * np.max(np.abs(rho))


# ------------------------------------------------ operator invariants


@pytest.mark.parametrize("cellname", list(CELLS))
def test_operator_invariants(oracle_mod, cellname):
    cell = CELLS[cellname].reshape(9)
    dims = (12, 10, 16)  # all even: Nyquist planes on every axis
    a = inputs.random_grid(dims, 1)
    b = inputs.random_grid(dims, 2)
    Pa, _, _, mia = oracle_mod.poisson(cell, a)
    Pb, _, _, mib = oracle_mod.poisson(cell, b)
    scale = np.linalg.norm(a) * np.linalg.norm(Pb)
    # symmetry <a, P b> = <P a, b>; the Nyquist reading keeps it for triclinic cells
    assert abs(np.vdot(a, Pb) - np.vdot(Pa, b)) <= 1e-13 * scale
    assert mia <= 1e-13 * np.max(np.abs(Pa)) and mib <= 1e-13 * np.max(np.abs(Pb))
    # positive semi-definite
    assert np.vdot(a, Pa) > 0
    # constants are in the null space, and V has zero mean
    P1, _, _, _ = oracle_mod.poisson(cell, np.ones(dims))
    assert np.max(np.abs(P1)) <= 1e-13
    assert abs(Pa.mean()) <= 1e-13 * np.max(np.abs(Pa))
    # a shift by grid vectors shifts V
    Ps, _, _, _ = oracle_mod.poisson(cell, np.roll(a, (3, -2, 5), axis=(0, 1, 2)))
    assert np.max(np.abs(Ps - np.roll(Pa, (3, -2, 5), axis=(0, 1, 2)))) <= 1e-12 * np.max(np.abs(Pa))


def test_kernel_symmetry_triclinic(oracle_mod):
    """K(m) = K(-m) on every index, Nyquist included."""
    cell = CELLS["triclinic"].reshape(9)
    for dims in [(8, 6, 10), (9, 6, 4), (2, 4, 6)]:
        K = oracle_mod.kernel(cell, dims)
        Km = K[np.ix_(*[(-np.arange(n)) % n for n in dims])]
        assert np.max(np.abs(K - Km)) <= 1e-15 * np.max(K)
        assert K[0, 0, 0] == 0.0


def test_cell_scaling(oracle_mod):
    """Scaling the cell by s at fixed grid values: V -> s^2 V, E_H -> s^5 E_H."""
    cell = CELLS["triclinic"]
    rho = inputs.random_grid((10, 12, 9), 4)
    V1, e1, _, _ = oracle_mod.poisson(cell.reshape(9), rho)
    s = 1.7
    V2, e2, _, _ = oracle_mod.poisson((s * cell).reshape(9), rho)
    assert np.max(np.abs(V2 - s * s * V1)) <= 1e-13 * np.max(np.abs(V2))
    assert abs(e2 - s ** 5 * e1) <= 1e-13 * abs(e2)


# --------------------------------------------------- backward


@pytest.mark.parametrize("cellname", ["ortho", "triclinic"])
def test_backward_directional_derivative(oracle_mod, cellname):
    """L(rho) = gE * E_H + <c, V>; L is quadratic, so the central difference
    along any direction equals <grad, direction> up to rounding."""
    cell = CELLS[cellname].reshape(9)
    dims = (10, 12, 8)
    rho = inputs.random_grid(dims, 20)
    c = inputs.random_grid(dims, 21)
    d = inputs.random_grid(dims, 22)
    gE = 0.7

    def loss(x):
        V, e, _, _ = oracle_mod.poisson(cell, x)
        return gE * e + float(np.vdot(c, V))

    g = oracle_mod.backward(cell, rho, grad_v=c, grad_e=gE)
    eps = 1e-3
    fd = (loss(rho + eps * d) - loss(rho - eps * d)) / (2 * eps)
    assert abs(fd - np.vdot(g, d)) <= 1e-10 * abs(fd)
    # no upstream gradient on V: grad = gE dV P rho
    g2 = oracle_mod.backward(cell, rho, grad_v=None, grad_e=1.0)
    V, _, _, _ = oracle_mod.poisson(cell, rho)
    dv = abs(np.linalg.det(cell.reshape(3, 3))) / rho.size
    assert np.max(np.abs(g2 - dv * V)) <= 1e-13 * np.max(np.abs(dv * V))


# ------------------------------------------------ Gaussians: splat


def brute_splat(cell, dims, pos, Z, sigma, nimg=2):
    """Per-point sum over explicit lattice images n in [-nimg, nimg]^3."""
    r = grid_points(cell, dims).reshape(-1, 3)
    out = np.zeros(r.shape[0])
    rng = range(-nimg, nimg + 1)
    imgs = np.array([[i, j, k] for i in rng for j in rng for k in rng], float) @ np.asarray(cell, float)
    for R, z, s in zip(pos, Z, sigma):
        d = r[:, None, :] - (R[None, None, :] + imgs[None, :, :])
        out += z * (2 * np.pi * s * s) ** -1.5 * np.exp(-np.sum(d * d, -1) / (2 * s * s)).sum(1)
    return out.reshape(dims)


@pytest.mark.parametrize("cellname", ["ortho", "triclinic"])
def test_splat_vs_brute_force(oracle_mod, cellname):
    cell = CELLS[cellname]
    dims = (10, 9, 12)
    rng = np.random.default_rng(3)
    pos = rng.random((3, 3)) @ cell + np.array([[0.0, 0.0, 0.0], [-3.0, 0.5, 0.2], [0.0, 0.0, 20.0]])
    Z = np.array([4.0, 1.0, 6.0])
    sigma = np.array([0.8, 1.3, 0.6])
    ref = brute_splat(cell, dims, pos, Z, sigma, nimg=3)
    got = oracle_mod.splat(cell.reshape(9), dims, pos, Z, sigma, subtract_background=False)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(ref)
    flat = np.array([0, 7, 555, got.size - 1])
    pts = oracle_mod.splat_points(cell.reshape(9), dims, pos, Z, sigma, flat, subtract_background=False)
    assert np.max(np.abs(pts - got.reshape(-1)[flat])) <= 1e-13 * np.max(ref)


def test_splat_total_charge(oracle_mod):
    """Sum rho dV = Q without background, 0 with it (Poisson summation; the
    grid error is ~exp(-2 pi^2 sigma^2 / h^2), far below 1e-13 here)."""
    p = inputs.cubic32()
    cell = p.cell.reshape(9)
    omega = abs(np.linalg.det(p.cell))
    dv = omega / p.npoints
    rho = oracle_mod.splat(cell, p.dims, p.pos, p.Z, p.sigma, subtract_background=False)
    assert abs(rho.sum() * dv - p.Z.sum()) <= 1e-12 * p.Z.sum()
    rho0 = oracle_mod.splat(cell, p.dims, p.pos, p.Z, p.sigma, subtract_background=True)
    assert abs(rho0.sum() * dv) <= 1e-12 * p.Z.sum()


# ---------------------------------------- Gaussians: energy and forces


def g_sum(cell, pos, Z, sigma, gmax_sigma=9.0):
    """Direct reciprocal-space sums for periodic Gaussians (numpy only):
    E = (2 pi / Omega) sum_{G != 0} |S(G)|^2 / |G|^2, and dE/dR."""
    B = recip_np(cell)
    omega = abs(np.linalg.det(cell))
    gmax = gmax_sigma / np.min(sigma)
    mmax = [int(np.ceil(gmax * np.linalg.norm(cell[d]) / (2 * np.pi))) + 1 for d in range(3)]
    m = np.stack(np.meshgrid(*[np.arange(-k, k + 1) for k in mmax], indexing="ij"), -1).reshape(-1, 3)
    m = m[np.any(m != 0, 1)]
    G = m @ B
    g2 = np.sum(G * G, 1)
    keep = g2 <= gmax * gmax
    G, g2 = G[keep], g2[keep]
    form = Z[:, None] * np.exp(-0.5 * sigma[:, None] ** 2 * g2[None, :])      # (n, nG)
    ph = np.exp(-1j * (pos @ G.T))                                           # (n, nG)
    S = np.sum(form * ph, 0)
    E = 2 * np.pi / omega * np.sum(np.abs(S) ** 2 / g2)
    im = np.imag(np.conj(S)[None, :] * ph)                                   # (n, nG)
    dE = 4 * np.pi / omega * ((form * im / g2[None, :]) @ G)
    return E, dE


def test_single_gaussian_ewald_closed_form(oracle_mod):
    """One Gaussian (Z=4, sigma=0.8) in a simple-cubic cell of edge 10 Bohr:
    E_H = Z^2 [1/(2 sigma sqrt(pi)) - alpha/(2L) + 2 pi sigma^2/L^3]
          - Z^2/2 sum_{n != 0} erfc(|nL| / 2 sigma) / |nL|."""
    Z, s, L = 4.0, 0.8, 10.0
    nr = 3
    n = np.array([[i, j, k] for i in range(-nr, nr + 1) for j in range(-nr, nr + 1)
                  for k in range(-nr, nr + 1) if (i, j, k) != (0, 0, 0)], float)
    d = np.linalg.norm(n * L, axis=1)
    e_cf = Z * Z * (1 / (2 * s * np.sqrt(np.pi)) - MADELUNG_SC / (2 * L) + 2 * np.pi * s * s / L ** 3) \
        - Z * Z / 2 * np.sum(erfc(d / (2 * s)) / d)
    cell = np.diag([L, L, L])
    pos = np.array([[3.1, 4.7, 8.2]])
    rho = oracle_mod.splat(cell.reshape(9), (32, 32, 32), pos, [Z], [s])
    V, e_real, e_recip, _ = oracle_mod.poisson(cell.reshape(9), rho)
    assert abs(e_recip - e_cf) <= 1e-12 * e_cf
    assert abs(e_real - e_cf) <= 1e-12 * e_cf


@pytest.mark.parametrize("which", ["cubic32", "small_mixed"])
def test_gaussian_energy_and_forces_vs_g_sum(oracle_mod, which):
    if which == "cubic32":
        p = inputs.cubic32()
    else:
        p = inputs.small_problem((36, 40, 45), 12, seed=9)
    cell9 = p.cell.reshape(9)
    rho = oracle_mod.splat(cell9, p.dims, p.pos, p.Z, p.sigma)
    V, e_real, e_recip, _ = oracle_mod.poisson(cell9, rho)
    E, dE = g_sum(p.cell, p.pos, p.Z, p.sigma)
    assert abs(e_recip - E) <= 1e-10 * E
    assert abs(e_real - E) <= 1e-10 * E
    dv = abs(np.linalg.det(p.cell)) / p.npoints
    grad = oracle_mod.splat_adjoint(cell9, p.pos, p.Z, p.sigma, dv * V)
    assert np.max(np.abs(grad - dE)) <= 1e-9 * np.max(np.abs(dE))
    # Newton's third law: the Hartree forces sum to zero
    assert np.max(np.abs(grad.sum(0))) <= 1e-9 * np.max(np.abs(dE))


def test_forces_vs_finite_differences(oracle_mod):
    p = inputs.small_problem((30, 30, 30), 6, seed=17, L=(8.0, 8.5, 9.0))
    cell9 = p.cell.reshape(9)

    def energy(pos):
        rho = oracle_mod.splat(cell9, p.dims, pos, p.Z, p.sigma)
        return oracle_mod.poisson(cell9, rho)[2]

    rho = oracle_mod.splat(cell9, p.dims, p.pos, p.Z, p.sigma)
    V = oracle_mod.poisson(cell9, rho)[0]
    dv = abs(np.linalg.det(p.cell)) / p.npoints
    grad = oracle_mod.splat_adjoint(cell9, p.pos, p.Z, p.sigma, dv * V)
    h = 1e-4
    for a in (0, 3):
        for x in range(3):
            dp = np.zeros_like(p.pos)
            dp[a, x] = h
            fd = (energy(p.pos + dp) - energy(p.pos - dp)) / (2 * h)
            assert abs(fd - grad[a, x]) <= 1e-5, (a, x, fd, grad[a, x])


def test_adjoint_selection_matches_full(oracle_mod):
    p = inputs.small_problem((20, 24, 18), 9, seed=2)
    cell9 = p.cell.reshape(9)
    g = inputs.random_grid(p.dims, 5)
    full = oracle_mod.splat_adjoint(cell9, p.pos, p.Z, p.sigma, g)
    sel = np.array([7, 0, 3])
    part = oracle_mod.splat_adjoint(cell9, p.pos, p.Z, p.sigma, g, sel=sel)
    assert np.array_equal(part, full[sel])


def test_rejects_bad_arguments(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.poisson(np.zeros(9), np.ones((4, 4, 4)))
    with pytest.raises(ValueError):
        oracle_mod.splat(np.eye(3).reshape(9), (4, 4, 4), [[0, 0, 0]], [1.0], [-1.0])
