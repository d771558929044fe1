"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Every test prints the case it is about to run before touching the GPU.
Tolerances: FP64 V rel-L2 <= 1e-12, E_H rel <= 1e-12, density max-rel <= 1e-13
(of the largest value), forces max-rel <= 1e-10; FP32 V rel-L2 <= 5e-6, E_H
rel <= 1e-6, density max-rel <= 1e-6, forces max-rel <= 1e-5.  The FP32
inputs are rounded to float first and the oracle is fed the same rounded
values.
"""
import itertools

import numpy as np
import pytest
import torch

from paper_1209_4506_amd import inputs

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a HIP device")]

TOL = {"fp64": dict(v=1e-12, e=1e-12), "fp32": dict(v=5e-6, e=1e-6)}
CELLS = {
    "cubic": np.diag([10.0, 10.0, 10.0]),
    "ortho": np.diag([8.0, 11.0, 13.5]),
    "triclinic": np.array([[9.0, 0.0, 0.0], [2.5, 8.0, 0.0], [-1.5, 2.0, 10.5]]),
}
# several tiles, ragged tails, odd and even Nc, radix 7, a degenerate axis, and
# every length class up to 1024 on some axis
DIMS = [(12, 10, 15), (32, 32, 32), (45, 36, 40), (7, 14, 21), (1, 6, 10), (50, 48, 27), (64, 60, 90),
        (36, 40, 360), (20, 300, 24), (270, 12, 16), (1024, 4, 6), (6, 1024, 4), (4, 6, 1024), (2, 2, 2), (1, 1, 1)]


def say(*a):
    print(*a, flush=True)


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def to_dev(x, dtype):
    return torch.tensor(np.ascontiguousarray(x), device="cuda", dtype=dtype)


@pytest.fixture(scope="module")
def H():
    import paper_1209_4506_amd.hartree as h

    return h


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("cellname", ["ortho", "triclinic"])
def test_solve_parity(H, oracle_mod, prec, dims, cellname):
    say("case solve", prec, dims, cellname)
    cell = CELLS[cellname]
    plan = H.Plan(cell, dims, precision=prec, max_atoms=1)
    rho = inputs.random_grid(dims, 7).astype(np.float32 if prec == "fp32" else np.float64)
    V, E = plan.solve(to_dev(rho, plan.dtype))
    e_only = plan.energy(to_dev(rho, plan.dtype))
    torch.cuda.synchronize()
    V_o, e_real, e_recip, _ = oracle_mod.poisson(cell.reshape(9), rho.astype(np.float64))
    ev = rel_l2(V.double().cpu().numpy(), V_o)
    ee = abs(float(E[0]) - e_recip) / max(abs(e_recip), 1e-300)
    say("  V rel-L2 %.3e  E_H rel %.3e" % (ev, ee))
    assert ev <= TOL[prec]["v"]
    if np.prod(dims) > 1:
        assert ee <= TOL[prec]["e"]
    else:
        assert float(E[0]) == 0.0 and e_recip == 0.0
    # the energy-only pass sums the same partials in the same order
    assert float(e_only[0]) == float(E[0])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dims", [(12, 10, 15), (45, 36, 40), (36, 40, 360)])
def test_backward_parity(H, oracle_mod, prec, dims):
    say("case backward", prec, dims)
    cell = CELLS["triclinic"]
    plan = H.Plan(cell, dims, precision=prec, max_atoms=1)
    ft = np.float32 if prec == "fp32" else np.float64
    rho = inputs.random_grid(dims, 1).astype(ft)
    gv = inputs.random_grid(dims, 2).astype(ft)
    ge = 0.7
    out = plan.backward(grad_v=to_dev(gv, plan.dtype), grad_e=torch.tensor([ge], dtype=torch.float64),
                        rho=to_dev(rho, plan.dtype))
    only_e = plan.backward(grad_v=None, grad_e=torch.tensor([ge], dtype=torch.float64), rho=to_dev(rho, plan.dtype))
    only_v = plan.backward(grad_v=to_dev(gv, plan.dtype))
    torch.cuda.synchronize()
    ref = oracle_mod.backward(cell.reshape(9), rho.astype(np.float64), grad_v=gv.astype(np.float64), grad_e=ge)
    ref_e = oracle_mod.backward(cell.reshape(9), rho.astype(np.float64), grad_v=None, grad_e=ge)
    ref_v = oracle_mod.backward(cell.reshape(9), rho.astype(np.float64), grad_v=gv.astype(np.float64), grad_e=0.0)
    for got, want, name in ((out, ref, "both"), (only_e, ref_e, "grad_e"), (only_v, ref_v, "grad_v")):
        r = rel_l2(got.double().cpu().numpy(), want)
        say("  %s rel-L2 %.3e" % (name, r))
        assert r <= TOL[prec]["v"]


def _atoms(p, dev="cuda"):
    return (torch.tensor(p.pos, device=dev), torch.tensor(p.Z, device=dev), torch.tensor(p.sigma, device=dev))


SPLAT_CASES = {
    "cubic32": lambda: inputs.cubic32(),
    # edges of 8-9 Bohr with sigma up to 1: at 8 sigma the truncation window is
    # wider than the cell, so several periodic images meet on one grid point
    "tight_images": lambda: inputs.small_problem((30, 36, 40), 20, seed=3, L=(8.0, 8.5, 9.0)),
    "ragged": lambda: inputs.small_problem((45, 27, 50), 37, seed=4, L=(12.0, 7.5, 14.0), sig=(0.6, 0.9)),
    # general (non-diagonal) cells: the direct-evaluation kernels
    "triclinic": lambda: inputs.small_cell_problem(CELLS["triclinic"], (36, 32, 40), 30, seed=5),
    "triclinic_tight": lambda: inputs.small_cell_problem(
        np.array([[7.0, 0.0, 0.0], [2.0, 7.5, 0.0], [-1.5, 1.0, 8.0]]), (28, 30, 35), 14, seed=6),
}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", list(SPLAT_CASES))
def test_splat_parity(H, oracle_mod, prec, case):
    say("case splat", prec, case)
    p = SPLAT_CASES[case]()
    plan = H.Plan(p.cell, p.dims, precision=prec, max_atoms=p.natoms)
    pos, Z, sig = _atoms(p)
    rho = plan.splat(pos, Z, sig).double().cpu().numpy()
    rho_nb = plan.splat(pos, Z, sig, subtract_background=False).double().cpu().numpy()
    assert plan.device_status() == 0
    ref = oracle_mod.splat(p.cell.reshape(9), p.dims, p.pos, p.Z, p.sigma)
    ref_nb = oracle_mod.splat(p.cell.reshape(9), p.dims, p.pos, p.Z, p.sigma, subtract_background=False)
    scale = np.abs(ref_nb).max()
    e1 = np.abs(rho - ref).max() / scale
    e2 = np.abs(rho_nb - ref_nb).max() / scale
    say("  rho max-rel %.3e (background) %.3e (none)" % (e1, e2))
    tol = 1e-13 if prec == "fp64" else 1e-6
    assert e1 <= tol and e2 <= tol


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", list(SPLAT_CASES))
def test_splat_adjoint_parity(H, oracle_mod, prec, case):
    say("case adjoint", prec, case)
    p = SPLAT_CASES[case]()
    plan = H.Plan(p.cell, p.dims, precision=prec, max_atoms=p.natoms)
    pos, Z, sig = _atoms(p)
    # a smooth field: the Hartree potential of the atoms themselves
    rho_o = oracle_mod.splat(p.cell.reshape(9), p.dims, p.pos, p.Z, p.sigma)
    V_o = oracle_mod.poisson(p.cell.reshape(9), rho_o)[0]
    g = V_o.astype(np.float32 if prec == "fp32" else np.float64)
    got = plan.splat_adjoint(pos, Z, sig, to_dev(g, plan.dtype)).cpu().numpy()
    assert plan.device_status() == 0
    ref = oracle_mod.splat_adjoint(p.cell.reshape(9), p.pos, p.Z, p.sigma, g.astype(np.float64))
    err = np.abs(got - ref).max() / np.abs(ref).max()
    say("  grad max-rel %.3e" % err)
    assert err <= (1e-10 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_many_atoms_one_problem(H, oracle_mod, prec):
    """33,000 atoms in one problem, more than the binning's bitmap ranks cover
    (32,768 atoms per problem): the brick lists are then ranked by counting.
    The density at sampled points and the forces on 8 seeded atoms against the
    oracle; two splats agree bit for bit."""
    say("case many atoms in one problem", prec)
    p = inputs.small_problem((192, 192, 96), 33000, seed=12, L=(60.0, 60.0, 30.0), sig=(0.6, 0.7))
    cell9 = p.cell.reshape(9)
    plan = H.Plan(p.cell, p.dims, precision=prec, max_atoms=p.natoms)
    pos, Z, sig = _atoms(p)
    rho = plan.splat(pos, Z, sig)
    rho2 = plan.splat(pos, Z, sig)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    assert torch.equal(rho, rho2)
    rng = np.random.default_rng(12)
    flat = rng.choice(int(np.prod(p.dims)), 100, replace=False)
    ref = oracle_mod.splat_points(cell9, p.dims, p.pos, p.Z, p.sigma, flat)
    got = rho.reshape(-1)[torch.tensor(flat, device="cuda")].double().cpu().numpy()
    err = np.abs(got - ref).max() / float(torch.max(torch.abs(rho)).item())
    say("  sampled density max-rel %.3e" % err)
    assert err <= (1e-13 if prec == "fp64" else 1e-6)
    # a smooth field for the adjoint
    ix = [np.arange(n) / n for n in p.dims]
    g = (np.cos(2 * np.pi * ix[0])[:, None, None] + 0.5 * np.sin(4 * np.pi * ix[1])[None, :, None]
         + 0.25 * np.cos(2 * np.pi * ix[2])[None, None, :]).astype(np.float32 if prec == "fp32" else np.float64)
    F = plan.splat_adjoint(pos, Z, sig, to_dev(g, plan.dtype)).cpu().numpy()
    assert plan.device_status() == 0
    sel = rng.choice(p.natoms, 8, replace=False)
    ref = oracle_mod.splat_adjoint(cell9, p.pos, p.Z, p.sigma, g.astype(np.float64), sel=sel)
    err = np.abs(F[sel] - ref).max() / np.abs(ref).max()
    say("  forces on 8 atoms max-rel %.3e" % err)
    assert err <= (1e-10 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_end_to_end_cubic32(H, oracle_mod, prec):
    """32^3 cubic cell, 8 Gaussians: splat, V, E_H, and dL/dR for
    L = E_H + <c, V> dV, all against the oracle."""
    say("case end-to-end cubic32", prec)
    p = inputs.cubic32()
    cell9 = p.cell.reshape(9)
    plan = H.Plan(p.cell, p.dims, precision=prec, max_atoms=p.natoms)
    pos, Z, sig = _atoms(p)
    pos.requires_grad_(True)
    V, E = H.hartree(pos, Z, sig, plan)
    c = inputs.random_grid(p.dims, 99)
    dv = plan.dv()[0]
    L = E.sum() + (V.double() * to_dev(c, torch.float64)).sum() * dv
    L.backward()
    torch.cuda.synchronize()
    rho_o = oracle_mod.splat(cell9, p.dims, p.pos, p.Z, p.sigma)
    V_o, _, E_o, _ = oracle_mod.poisson(cell9, rho_o)
    g_o = oracle_mod.backward(cell9, rho_o, grad_v=c * dv, grad_e=1.0)
    gp_o = oracle_mod.splat_adjoint(cell9, p.pos, p.Z, p.sigma, g_o)
    ev = rel_l2(V.detach().double().cpu().numpy(), V_o)
    ee = abs(float(E[0]) - E_o) / E_o
    ef = np.abs(pos.grad.cpu().numpy() - gp_o).max() / np.abs(gp_o).max()
    say("  V %.3e  E_H %.3e  grad %.3e" % (ev, ee, ef))
    assert ev <= TOL[prec]["v"] and ee <= TOL[prec]["e"]
    assert ef <= (1e-10 if prec == "fp64" else 1e-5)


def test_bitwise_reproducible(H):
    say("case reproducible diamond180 fp32")
    p = inputs.diamond180()
    plan = H.Plan(p.cell, p.dims, precision="fp32", max_atoms=p.natoms)
    pos, Z, sig = _atoms(p)
    outs = []
    for _ in range(2):
        rho = plan.splat(pos, Z, sig)
        V, E = plan.solve(rho)
        g = plan.backward(grad_v=V, grad_e=torch.ones(1, dtype=torch.float64), rho=rho)
        f = plan.splat_adjoint(pos, Z, sig, g)
        outs.append([rho.cpu(), V.cpu(), E.cpu(), g.cpu(), f.cpu()])
    for a, b in zip(*outs):
        assert torch.equal(a, b)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("mode", ["bisection", "shuffled"])
def test_atom_order_equivariance(H, prec, mode):
    """The atoms in another order (the recursive-bisection order of
    hartree_atom_partition, or a random one) give the same density and the
    same forces, permuted: only the rounding order of the sums may change."""
    say("case atom order", mode, prec, "diamond180")
    p = inputs.diamond180()
    if mode == "bisection":
        perm = H.atom_partition(p.pos, 16)[0].astype(np.int64)
    else:
        perm = np.random.default_rng(17).permutation(p.natoms)
    plan = H.Plan(p.cell, p.dims, precision=prec, max_atoms=p.natoms)
    g = to_dev(inputs.random_grid(p.dims, 23), plan.dtype)
    res = []
    for idx in (np.arange(p.natoms), perm):
        pos = torch.tensor(p.pos[idx], device="cuda")
        Z = torch.tensor(p.Z[idx], device="cuda")
        sig = torch.tensor(p.sigma[idx], device="cuda")
        tok = plan.bind_atoms(pos, Z, sig)
        rho = plan.splat_bound(tok).double().cpu().numpy()
        f = plan.splat_adjoint_bound(tok, g).cpu().numpy()
        res.append((rho, f))
    assert plan.device_status() == 0
    (rho0, f0), (rho1, f1) = res
    back = np.empty_like(f1)
    back[perm] = f1
    er = np.abs(rho1 - rho0).max() / np.abs(rho0).max()
    ef = np.abs(back - f0).max() / np.abs(f0).max()
    say("  rho max-rel %.3e  grad max-rel %.3e" % (er, ef))
    assert er <= (1e-13 if prec == "fp64" else 1e-6)
    assert ef <= (1e-11 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("fill", [0x00, 0xFF])
def test_workspace_contents_do_not_matter(H, oracle_mod, prec, fill):
    """A workspace handed over full of arbitrary bytes gives the same bits as
    any other: every kernel writes what it reads (the binding clears the
    parts that must start at zero).  Regression: the per-atom table pass
    once ran before the pass that prepares the atoms."""
    say("case workspace filled with 0x%02x" % fill, prec)
    outs = []
    for case in ("ragged", "tight_images"):
        p = SPLAT_CASES[case]()
        plan = H.Plan(p.cell, p.dims, precision=prec, max_atoms=p.natoms, bind=False)
        need = plan.workspace_size()
        raw = torch.full((need + 256,), fill, dtype=torch.uint8, device="cuda")
        shift = (-raw.data_ptr()) % 256
        plan.bind(raw[shift:shift + need])
        pos, Z, sig = _atoms(p)
        g = to_dev(inputs.random_grid(p.dims, 31), plan.dtype)
        rho = plan.splat(pos, Z, sig)
        V, E = plan.solve(rho)
        f = plan.splat_adjoint(pos, Z, sig, g)
        torch.cuda.synchronize()
        assert plan.device_status() == 0
        outs.append([rho.cpu(), V.cpu(), E.cpu(), f.cpu()])
        ref = oracle_splat_cache(oracle_mod, p)
        assert np.abs(rho.double().cpu().numpy() - ref).max() / np.abs(ref).max() <= (1e-13 if prec == "fp64" else 1e-6)
    key = (prec,)
    if key in _WS_REF:
        for a, b in zip(sum(_WS_REF[key], []), sum(outs, [])):
            assert torch.equal(a, b)
    else:
        _WS_REF[key] = outs


_WS_REF = {}
_SPLAT_REF = {}


def oracle_splat_cache(oracle_mod, p):
    key = (p.name, p.seed, p.dims)
    if key not in _SPLAT_REF:
        _SPLAT_REF[key] = oracle_mod.splat(p.cell.reshape(9), p.dims, p.pos, p.Z, p.sigma)
    return _SPLAT_REF[key]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", ["cubic32", "ragged", "tight_images"])
def test_binding_pairs(H, prec, case):
    """hartree_atoms_pairs equals the number of (atom, brick) pairs that the
    truncation windows define: per axis the bricks holding a grid index of
    [ceil((X - rc) / h), floor((X + rc) / h)] taken modulo the axis length
    (bricks of 16 x 16 x 32 points in both precisions for these diagonal
    cells)."""
    say("case binding pairs", prec, case)
    p = SPLAT_CASES[case]()
    plan = H.Plan(p.cell, p.dims, precision=prec, max_atoms=p.natoms)
    pos, Z, sig = _atoms(p)
    plan.bind_atoms(pos, Z, sig)
    got = plan.atoms_pairs()
    bsz = (16, 16, 32)
    rc_sig = 6.0 if prec == "fp32" else 8.0
    L = np.diag(p.cell)
    want = 0
    for i in range(p.natoms):
        cnt = 1
        for x in range(3):
            n, h = p.dims[x], L[x] / p.dims[x]
            X = p.pos[i, x] % L[x]
            rc = rc_sig * p.sigma[i]
            lo, hi = int(np.ceil((X - rc) / h)), int(np.floor((X + rc) / h))
            cnt *= len({(g % n) // bsz[x] for g in range(lo, hi + 1)})
        want += cnt
    assert got == want


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_zero_atoms(H, prec):
    """No atoms: the density is zero (no charge, no background), the binding
    is empty, and the adjoint has nothing to write."""
    say("case zero atoms", prec)
    plan = H.Plan(np.eye(3) * 9.0, (24, 30, 36), precision=prec, max_atoms=4)
    e = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    z = torch.zeros(0, dtype=torch.float64, device="cuda")
    rho = plan.splat(e, z, z)
    assert plan.atoms_pairs() == 0
    assert torch.count_nonzero(rho).item() == 0
    f = plan.splat_adjoint(e, z, z, torch.ones_like(rho))
    assert f.shape == (0, 3)
    V, E = plan.solve(rho)
    assert torch.count_nonzero(V).item() == 0 and float(E[0]) == 0.0
    assert plan.device_status() == 0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", ["ragged", "triclinic", "tight_images"])
def test_periodic_images_of_atoms(H, prec, case):
    """Atoms given anywhere in space (shifted by whole cell vectors, also
    negative) give the density and forces of their images in the cell."""
    say("case periodic images", prec, case)
    p = SPLAT_CASES[case]()
    plan = H.Plan(p.cell, p.dims, precision=prec, max_atoms=p.natoms)
    rng = np.random.default_rng(19)
    shifts = rng.integers(-3, 4, size=(p.natoms, 3)) @ p.cell
    g = to_dev(inputs.random_grid(p.dims, 29), plan.dtype)
    res = []
    for pos_np in (p.pos, p.pos + shifts):
        pos = torch.tensor(pos_np, device="cuda")
        Z = torch.tensor(p.Z, device="cuda")
        sig = torch.tensor(p.sigma, device="cuda")
        res.append((plan.splat(pos, Z, sig).double().cpu().numpy(), plan.splat_adjoint(pos, Z, sig, g).cpu().numpy()))
    assert plan.device_status() == 0
    (r0, f0), (r1, f1) = res
    er = np.abs(r1 - r0).max() / np.abs(r0).max()
    ef = np.abs(f1 - f0).max() / np.abs(f0).max()
    say("  rho max-rel %.3e  grad max-rel %.3e" % (er, ef))
    assert er <= (1e-13 if prec == "fp64" else 1e-6)
    assert ef <= (1e-10 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_invalid_atoms_reported(H, prec):
    """A non-finite position or a width <= 0 sets HARTREE_DEV_BAD_ATOM; such
    an atom touches no grid point and gets a zero force."""
    say("case invalid atoms", prec)
    p = inputs.cubic32()
    plan = H.Plan(p.cell, p.dims, precision=prec, max_atoms=p.natoms)
    for bad in ("pos", "sigma"):
        pos = torch.tensor(p.pos, device="cuda")
        Z = torch.tensor(p.Z, device="cuda")
        sig = torch.tensor(p.sigma, device="cuda")
        if bad == "pos":
            pos[3, 1] = float("nan")
        else:
            sig[3] = 0.0
        rho = plan.splat(pos, Z, sig)
        assert plan.device_status() & H.DEV_BAD_ATOM
        f = plan.splat_adjoint(pos, Z, sig, torch.ones_like(rho))
        assert plan.device_status() & H.DEV_BAD_ATOM
        assert torch.count_nonzero(f[3]).item() == 0
        assert torch.isfinite(f).all()


def test_rejects_arguments(H):
    say("case argument errors")
    with pytest.raises(H.HartreeError) as ei:
        H.Plan(np.eye(3) * 10, (32, 32, 33))
    assert ei.value.code == 2
    with pytest.raises(H.HartreeError) as ei:
        H.Plan(np.zeros((3, 3)), (8, 8, 8))
    assert ei.value.code == 3
    pos = torch.zeros((1, 3), dtype=torch.float64, device="cuda")
    one = torch.ones(1, dtype=torch.float64, device="cuda")
    tri = H.Plan(CELLS["triclinic"], (8, 8, 8), max_atoms=4)
    with pytest.raises(H.HartreeError) as ei:  # more atoms than the plan was sized for
        tri.splat(torch.zeros((5, 3), dtype=torch.float64, device="cuda"), torch.ones(5), torch.ones(5))
    assert ei.value.code == 1
    plan = H.Plan(np.eye(3) * 8, (8, 8, 8), max_atoms=4, max_sigma=1.0)
    with pytest.raises(H.HartreeError) as ei:
        plan.splat(torch.zeros((5, 3), dtype=torch.float64, device="cuda"), torch.ones(5), torch.ones(5))
    assert ei.value.code == 1
    # a width beyond max_sigma is caught on the device and reported by the status word
    plan.splat(pos, one, one * 2.0)
    assert plan.device_status() & H.DEV_SIGMA_RANGE
    assert plan.device_status() == 0


def test_bound_atoms_reuse(H):
    """A binding shared by splat and adjoint gives the unbound results bit for
    bit; a rebinding invalidates older tokens."""
    say("case bound atoms")
    p = inputs.small_problem((30, 36, 40), 20, seed=3, L=(8.0, 8.5, 9.0))
    plan = H.Plan(p.cell, p.dims, precision="fp32", max_atoms=p.natoms)
    pos, Z, sig = _atoms(p)
    rho_u = plan.splat(pos, Z, sig)
    g = torch.randn(p.dims, device="cuda", dtype=torch.float32)
    f_u = plan.splat_adjoint(pos, Z, sig, g)
    tok = plan.bind_atoms(pos, Z, sig)
    rho_b = plan.splat_bound(tok)
    f_b = plan.splat_adjoint_bound(tok, g)
    torch.cuda.synchronize()
    assert torch.equal(rho_u, rho_b) and torch.equal(f_u, f_b)
    tok2 = plan.bind_atoms(pos + 0.1, Z, sig)
    assert tok2 != tok
    with pytest.raises(H.HartreeError):
        plan.splat_bound(tok)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("n", [360, 180])
def test_every_compiled_plan(H, oracle_mod, prec, n):
    """Every compiled radix plan that factors n, at every tile width the
    plan accepts and pitch pads 0 and 1 (strided axes), on each axis in turn
    (the a, b and c passes; some tile shapes have kernels of their own): the
    solve and the backward (with grad_v and grad_e, and grad_e alone) match
    the oracle.  The tuner may pick any of
    these, so each is checked, not only the default choice."""
    cell = CELLS["triclinic"]
    ft = np.float32 if prec == "fp32" else np.float64
    checked = 0
    for x in range(3):
        dims = [12, 10, 14]
        dims[x] = n
        dims = tuple(dims)
        plan = H.Plan(cell, dims, precision=prec, max_atoms=1)
        base = plan.get_config()
        rho = inputs.random_grid(dims, 31 + x).astype(ft)
        gv = inputs.random_grid(dims, 41 + x).astype(ft)
        V_o, _, e_recip, _ = oracle_mod.poisson(cell.reshape(9), rho.astype(np.float64))
        G_o = oracle_mod.backward(cell.reshape(9), rho.astype(np.float64), grad_v=gv.astype(np.float64), grad_e=0.3)
        G_e = oracle_mod.backward(cell.reshape(9), rho.astype(np.float64), grad_v=None, grad_e=0.3)
        rho_d, gv_d = to_dev(rho, plan.dtype), to_dev(gv, plan.dtype)
        for pid, lp, pad in itertools.product(range(64), range(7), (0,) if x == 2 else (0, 1)):
            cfg = base.copy()
            cfg[0, x] = (pid, lp, pad)
            try:
                plan.set_config(cfg)
            except H.HartreeError:
                continue
            say("case compiled plan", prec, dims, "axis", x, "entry", pid, "p_log2", lp, "pad", pad)
            V, E = plan.solve(rho_d)
            g = plan.backward(grad_v=gv_d, grad_e=torch.tensor([0.3], dtype=torch.float64), rho=rho_d)
            ge = plan.backward(grad_v=None, grad_e=torch.tensor([0.3], dtype=torch.float64), rho=rho_d)
            torch.cuda.synchronize()
            assert rel_l2(V.double().cpu().numpy(), V_o) <= TOL[prec]["v"]
            assert abs(float(E[0]) - e_recip) <= TOL[prec]["e"] * abs(e_recip)
            assert rel_l2(g.double().cpu().numpy(), G_o) <= TOL[prec]["v"]
            assert rel_l2(ge.double().cpu().numpy(), G_e) <= TOL[prec]["v"]
            checked += 1
    # 360 and 180 each have several compiled plans, radix-6 ones among them
    assert checked >= 12


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_tuned_plan_parity(H, oracle_mod, prec):
    """After hartree_plan_tune (and a config round trip) the solve and the
    backward still match the oracle; a batched plan tunes per length."""
    cell = CELLS["ortho"]
    dims = (45, 36, 40)
    say("case tuned plan", prec, dims)
    plan = H.Plan(cell, dims, precision=prec, max_atoms=1)
    before = plan.get_config()
    after = plan.tune(reps=2)
    assert after.shape == before.shape
    plan.set_config(after)
    assert np.array_equal(plan.get_config(), after)
    rho = inputs.random_grid(dims, 11).astype(np.float32 if prec == "fp32" else np.float64)
    V, E = plan.solve(to_dev(rho, plan.dtype))
    torch.cuda.synchronize()
    V_o, _, e_recip, _ = oracle_mod.poisson(cell.reshape(9), rho.astype(np.float64))
    assert rel_l2(V.double().cpu().numpy(), V_o) <= TOL[prec]["v"]
    assert abs(float(E[0]) - e_recip) <= TOL[prec]["e"] * abs(e_recip)

    say("case tuned batched plan", prec)
    cells = np.stack([CELLS["ortho"], CELLS["cubic"], CELLS["ortho"]])
    bdims = np.array([(45, 36, 40), (32, 32, 32), (36, 45, 21)])
    bplan = H.Plan(cells, bdims, precision=prec, max_atoms=1)
    bplan.tune(reps=2)
    grids = [inputs.random_grid(tuple(d), 20 + i).astype(np.float32 if prec == "fp32" else np.float64)
             for i, d in enumerate(bdims)]
    Vb, Eb = bplan.solve(to_dev(np.concatenate([g.reshape(-1) for g in grids]), bplan.dtype))
    torch.cuda.synchronize()
    Vb = Vb.double().cpu().numpy()
    for i, g in enumerate(grids):
        V_o, _, e_recip, _ = oracle_mod.poisson(cells[i].reshape(9), g.astype(np.float64))
        o0, o1 = bplan.offsets[i], bplan.offsets[i + 1]
        assert rel_l2(Vb[o0:o1], V_o.reshape(-1)) <= TOL[prec]["v"]
        assert abs(float(Eb[i]) - e_recip) <= TOL[prec]["e"] * abs(e_recip)


# the compiled plan lengths up to 240 (the first 16 entries of the plan
# table), which one multi-plan launch per pass serves in batched FP32 plans
SMALL_LENGTHS = [32, 48, 60, 64, 72, 90, 96, 120, 128, 150, 160, 180, 192, 200, 210, 240]


def multi_auto_log2(n, x):
    """log2 of the size-adapted multi-plan tile width for length n on axis x:
    the most pencils (at most 64 along a and b, 32 along c) whose points stay
    within 4096 (a) or 2048 (b, c), at least 8 (a, b) or 4 (c)."""
    p, lo, target = (32, 4, 2048) if x == 2 else (64, 8, 4096 if x == 0 else 2048)
    while p > lo and p * n > target:
        p //= 2
    return p.bit_length() - 1


@pytest.mark.parametrize("lp_ab,lp_c", [(4, 2), (3, 3), ("auto", "auto")])
def test_multi_plan_launch(H, oracle_mod, lp_ab, lp_c):
    """A batched FP32 plan whose every problem takes a compiled plan of length
    <= 240 at one common tile width per axis (8 or 16 pencils along a and b,
    4 or 8 along c), or each at its
    length's size-adapted width, with no pitch pad, runs each pass as one
    launch whose workgroups pick their problem's plan: every listed plan on
    every axis, diagonal and triclinic cells, every tile shape.  The solve
    and the backward (with grad_v and grad_e, and grad_e alone) match the
    oracle for each problem."""
    probs = []
    for x in range(3):
        for i, n in enumerate(SMALL_LENGTHS):
            d = [32, 48, 60]
            d[x] = n
            d[(x + 1) % 3] = 48 if i % 2 else 32
            probs.append((tuple(d), "triclinic" if (i + x) % 3 == 0 else "ortho"))
    cells = np.stack([CELLS[c] for _, c in probs])
    dims = np.array([d for d, _ in probs])
    say("case multi-plan launch:", len(probs), "problems, tile widths (log2)", lp_ab, lp_c)
    plan = H.Plan(cells, dims, precision="fp32", max_atoms=1)
    cfg = plan.get_config()
    # along a and b the table's entries 0 .. 15 are the plans of these
    # lengths, in order; along c the entries 41, 42, 43 (no radix-16 stage)
    # stand for 48, 128 and 160
    entry = {n: i for i, n in enumerate(SMALL_LENGTHS)}
    entry_c = {**entry, 48: 41, 128: 42, 160: 43}
    for q, (d, _) in enumerate(probs):
        for x in range(3):
            lp = lp_ab if x < 2 else lp_c
            lp = multi_auto_log2(d[x], x) if lp == "auto" else lp
            cfg[q, x] = (entry[d[x]], lp, 0) if x < 2 else (entry_c[d[x]], lp, 0)
    plan.set_config(cfg)
    grids = [inputs.random_grid(d, 60 + q).astype(np.float32) for q, (d, _) in enumerate(probs)]
    gvs = [inputs.random_grid(d, 160 + q).astype(np.float32) for q, (d, _) in enumerate(probs)]
    rho_d = to_dev(np.concatenate([g.reshape(-1) for g in grids]), plan.dtype)
    gv_d = to_dev(np.concatenate([g.reshape(-1) for g in gvs]), plan.dtype)
    ge = torch.tensor([0.3 + 0.01 * q for q in range(len(probs))], dtype=torch.float64)
    V, E = plan.solve(rho_d)
    G = plan.backward(grad_v=gv_d, grad_e=ge, rho=rho_d)
    Ge = plan.backward(grad_v=None, grad_e=ge, rho=rho_d)
    torch.cuda.synchronize()
    V, G, Ge = (t.double().cpu().numpy() for t in (V, G, Ge))
    for q, (d, c) in enumerate(probs):
        cell = CELLS[c].reshape(9)
        rho = grids[q].astype(np.float64)
        V_o, _, e_recip, _ = oracle_mod.poisson(cell, rho)
        G_o = oracle_mod.backward(cell, rho, grad_v=gvs[q].astype(np.float64), grad_e=float(ge[q]))
        G_e = oracle_mod.backward(cell, rho, grad_v=None, grad_e=float(ge[q]))
        o0, o1 = plan.offsets[q], plan.offsets[q + 1]
        assert rel_l2(V[o0:o1], V_o.reshape(-1)) <= TOL["fp32"]["v"], (q, d, c)
        assert abs(float(E[q]) - e_recip) <= TOL["fp32"]["e"] * abs(e_recip), (q, d, c)
        assert rel_l2(G[o0:o1], G_o.reshape(-1)) <= TOL["fp32"]["v"], (q, d, c)
        assert rel_l2(Ge[o0:o1], G_e.reshape(-1)) <= TOL["fp32"]["v"], (q, d, c)


def test_multi_plan_launch_noalloc(H):
    """The multi-plan launches through hartree_solve_noalloc: a batched FP32
    plan with no workspace bound, every pass one launch with tiles sized per
    length, gives V and E_H of hartree_solve under the same configuration
    (rel-L2 <= 5e-6, E_H rel <= 1e-6: the no-allocation call generates its
    twiddles on the device)."""
    probs = [((48, 60, 72), "ortho"), ((60, 72, 90), "triclinic"), ((72, 90, 120), "ortho"),
             ((90, 120, 48), "ortho"), ((120, 48, 60), "triclinic")]
    cells = np.stack([CELLS[c] for _, c in probs])
    dims = np.array([d for d, _ in probs])
    say("case multi-plan launch, no-allocation solve:", len(probs), "problems")
    entry = {n: i for i, n in enumerate(SMALL_LENGTHS)}
    entry_c = {**entry, 48: 41, 128: 42, 160: 43}
    ref = H.Plan(cells, dims, precision="fp32", max_atoms=1)
    plan = H.Plan(cells, dims, precision="fp32", max_atoms=1, bind=False)
    cfg = ref.get_config()
    for q, (d, _) in enumerate(probs):
        for x in range(3):
            cfg[q, x] = (entry[d[x]] if x < 2 else entry_c[d[x]], multi_auto_log2(d[x], x), 0)
    ref.set_config(cfg)
    plan.set_config(cfg)
    rho = to_dev(np.concatenate([inputs.random_grid(d, 70 + q).astype(np.float32).reshape(-1)
                                 for q, (d, _) in enumerate(probs)]), ref.dtype)
    V_ref, E_ref = ref.solve(rho)
    V = torch.full_like(V_ref, float("nan"))
    E = torch.full((len(probs),), float("nan"), dtype=torch.float64, device="cuda")
    plan.solve_noalloc(rho, V, E)
    torch.cuda.synchronize()
    V_ref, V = V_ref.double().cpu().numpy(), V.double().cpu().numpy()
    for q in range(len(probs)):
        o0, o1 = ref.offsets[q], ref.offsets[q + 1]
        assert rel_l2(V[o0:o1], V_ref[o0:o1]) <= TOL["fp32"]["v"], q
        assert abs(float(E[q]) - float(E_ref[q])) <= TOL["fp32"]["e"] * abs(float(E_ref[q])), q
