"""Atom decomposition of Sec. 3.1 on the CPU.

Part 1 pins the oracle (oracle/partition.py) to what the paper and the
mathematics fix: the paper's 26-atom / 4-process example, closed forms of the
inertia tensor, brute-force maximality of F over the unit sphere, the atom
counts that follow from the bisection rule alone, invariances, balance bounds
and locality on the paper's 16,384-atom / 19-process diamond demo.

Part 2 compares the library's host partitioner (hartree_atom_partition, C++)
with the oracle: the order, the part of every atom and the part offsets are
integers and must agree exactly wherever the decomposition is unique; on
degenerate inputs (several equally good axes) only validity is checked.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import partition as op
from paper_1209_4506_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


def random_rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def cloud(n, seed, scales=(6.0, 3.0, 1.5)):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(n, 3)) * np.asarray(scales) @ random_rotation(rng).T + rng.normal(size=3) * 10


def counts_tree(m, n):
    """Part sizes that the bisection rule alone fixes for unit weights: a node
    of m atoms and n processes gives the ceil(n/2)-process child the integer
    nearest to m*ceil(n/2)/n (halves rounded up)."""
    if n == 1 or m == 0:
        return [m] + [0] * (n - 1)
    nl = (n + 1) // 2
    share = Fraction(m * nl, n)
    k = int(share + Fraction(1, 2))  # floor(share + 1/2)
    return counts_tree(k, nl) + counts_tree(m - k, n - nl)


def check_valid(order, part, start, natoms, nparts):
    assert sorted(order.tolist()) == list(range(natoms))
    assert start[0] == 0 and start[-1] == natoms and np.all(np.diff(start) >= 0)
    for p in range(nparts):
        assert np.all(part[order[start[p]:start[p + 1]]] == p)


# ------------------------------------------------------------ oracle pins


def test_paper_example_26_atoms_4_processes():
    g = json.load(open(os.path.join(HERE, "golden", "bisection_26_atoms_4_processes.json")))
    for seed in range(5):
        x = cloud(g["natoms"], seed)
        order, part, start = op.decompose(x, g["nprocesses"])
        sizes = np.diff(start).tolist()
        assert [sizes[0] + sizes[1], sizes[2] + sizes[3]] == g["root_children_atoms"]
        assert [sizes[0:2], sizes[2:4]] == g["leaf_atoms_per_child"]


def test_inertia_tensor_box_vertices():
    # 8 unit masses at (+-a, +-b, +-c): T = 8 diag(b^2+c^2, a^2+c^2, a^2+b^2)
    a, b, c = 1.5, 0.7, 2.2
    x = np.array([[sa * a, sb * b, sc * c] for sa in (-1, 1) for sb in (-1, 1) for sc in (-1, 1)]) + [3.0, -1.0, 2.0]
    w = np.ones(8)
    T = op.inertia_tensor(x, w, op.centre(x, w))
    np.testing.assert_allclose(T, 8 * np.diag([b * b + c * c, a * a + c * c, a * a + b * b]), atol=1e-12)


def test_inertia_tensor_two_masses_reduced_mass():
    # two masses: T = mu (|d|^2 I - d d^T), mu = w1 w2 / (w1 + w2), about their weighted centre
    p1, p2 = np.array([1.0, -2.0, 0.5]), np.array([4.0, 1.0, -1.5])
    w = np.array([0.3, 1.7])
    x = np.stack([p1, p2])
    d = p1 - p2
    mu = w[0] * w[1] / w.sum()
    T = op.inertia_tensor(x, w, op.centre(x, w))
    np.testing.assert_allclose(T, mu * (d @ d * np.eye(3) - np.outer(d, d)), rtol=1e-13, atol=1e-13)


def test_inertia_tensor_plane_and_rotation():
    rng = np.random.default_rng(3)
    x = np.c_[rng.normal(size=(50, 2)) * [2.0, 1.0], np.zeros(50)]
    w = rng.uniform(0.2, 1.0, 50)
    T = op.inertia_tensor(x, w, op.centre(x, w))
    assert T[2, 2] == pytest.approx(T[0, 0] + T[1, 1], rel=1e-13)  # perpendicular-axis theorem
    Q = random_rotation(rng)
    xr = x @ Q.T
    Tr = op.inertia_tensor(xr, w, op.centre(xr, w))
    np.testing.assert_allclose(Tr, Q @ T @ Q.T, atol=1e-11)  # a second-rank tensor
    ev = np.linalg.eigvalsh(T)
    assert ev[2] <= ev[0] + ev[1] + 1e-12  # triangle inequality of principal moments


def test_principal_axis_is_the_long_axis_and_maximises_F():
    rng = np.random.default_rng(4)
    u = rng.normal(size=3)
    u /= np.linalg.norm(u)
    x = np.outer(rng.normal(size=400) * 10.0, u) + rng.normal(size=(400, 3))
    w = rng.uniform(0.1, 1.0, 400)
    c, a = op.principal_axis(x, w)
    assert abs(a @ u) > 0.999
    assert np.max(np.abs(a)) == a[np.argmax(np.abs(a))]  # sign convention
    # brute force over the sphere: no direction gives a larger F
    dirs = rng.normal(size=(20000, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    X = x - c
    Fs = ((X @ dirs.T) ** 2 * w[:, None]).sum(0)
    assert op.objective(x, w, c, a) >= Fs.max() * (1 - 1e-12)


def test_lower_parts_hold_the_lower_projections():
    # documented convention: part 0 .. ceil(n/2)-1 lie below the split plane
    # along the axis whose largest component is positive
    x = cloud(500, 9)
    w = np.random.default_rng(9).uniform(0.1, 1.0, 500)
    order, part, start = op.decompose(x, 3, w)
    c, a = op.principal_axis(x, w)
    t = op.projection(x, c, a)
    assert a[np.argmax(np.abs(a))] > 0
    assert t[part <= 1].max() <= t[part == 2].min()


def test_split_index_is_nearest_with_ties_to_the_lower_child():
    assert op.split_index(np.ones(13), 1, 2) == 7
    assert op.split_index(np.ones(1), 1, 2) == 1
    assert op.split_index(np.ones(3), 2, 3) == 2
    rng = np.random.default_rng(5)
    for _ in range(200):
        m = int(rng.integers(1, 30))
        n = int(rng.integers(2, 12))
        ws = rng.uniform(0.05, 1.0, m)
        nl = (n + 1) // 2
        k = op.split_index(ws, nl, n)
        target = ws.sum() * nl / n
        errs = [abs(ws[:j].sum() - target) for j in range(m + 1)]
        assert errs[k] <= min(errs) + 1e-12
        assert errs[k] <= ws.max() / 2 + 1e-12


@pytest.mark.parametrize("natoms,nparts", [(26, 4), (16384, 19), (1000, 7), (5, 8), (0, 3), (1, 1), (3, 19), (100, 64)])
def test_unit_weight_sizes_follow_the_count_tree(natoms, nparts):
    x = cloud(natoms, 11 + natoms)
    order, part, start = op.decompose(x, nparts)
    check_valid(order, part, start, natoms, nparts)
    assert np.diff(start).tolist() == counts_tree(natoms, nparts)


def test_invariances():
    rng = np.random.default_rng(6)
    x = cloud(700, 6)
    w = rng.uniform(0.1, 1.0, 700)
    ref = op.decompose(x, 11, w)
    # translation (the centre is normalised by the total weight)
    got = op.decompose(x + np.array([40.0, -17.0, 3.0]), 11, w)
    assert all(np.array_equal(a, b) for a, b in zip(ref, got))
    # rotation: the axis sign may flip with the frame, which mirrors the
    # order; with 2^k processes every split halves the weight, so the parts
    # themselves (as sets of atoms) are unchanged
    def parts(res):
        order, _, start = res
        return {frozenset(order[start[p]:start[p + 1]].tolist()) for p in range(len(start) - 1)}

    ref8 = op.decompose(x, 8, w)
    for _ in range(3):
        assert parts(op.decompose(x @ random_rotation(rng).T, 8, w)) == parts(ref8)
    # scaling every weight (Eq. (19) normalises by the longest time)
    got = op.decompose(x, 11, w * 3.7)
    assert np.array_equal(ref[1], got[1])


def test_weight_balance():
    rng = np.random.default_rng(7)
    x = cloud(3000, 7)
    w = rng.uniform(0.05, 1.0, 3000)
    order, part, start = op.decompose(x, 2, w)
    lo = w[order[:start[1]]].sum()
    assert abs(lo - w.sum() / 2) <= w.max() / 2 + 1e-9
    order, part, start = op.decompose(x, 19, w)
    sums = np.array([w[order[start[p]:start[p + 1]]].sum() for p in range(19)])
    depth = int(np.ceil(np.log2(19)))
    assert np.all(np.abs(sums - w.sum() / 19) <= depth * w.max())


def test_heavy_atoms_weight_shifts_the_split():
    # atoms on a line, the first 20 four times heavier: the weight, not the
    # count, is halved (13 heavy atoms below, or 20 light + 8 heavy)
    x = np.c_[np.arange(40.0), np.zeros(40), np.zeros(40)] + np.random.default_rng(8).normal(0, 0.01, (40, 3))
    w = np.where(np.arange(40) < 20, 1.0, 0.25)
    order, part, start = op.decompose(x, 2, w)
    lower = set(order[:start[1]].tolist())
    assert abs(w[list(lower)].sum() - w.sum() / 2) <= 0.5
    assert len(lower) in (13, 28)


def test_diamond_16384_atoms_19_processes_locality():
    p = inputs.diamond16384()
    order, part, start = op.decompose(p.pos, 19)
    check_valid(order, part, start, p.natoms, 19)
    sizes = np.diff(start)
    assert sizes.min() >= 862 and sizes.max() <= 863
    rg = np.mean([np.sqrt(((p.pos[part == k] - p.pos[part == k].mean(0)) ** 2).sum(1).mean()) for k in range(19)])
    vol = abs(np.linalg.det(p.cell)) / 19
    rg_sphere = np.sqrt(3.0 / 5.0) * (3 * vol / (4 * np.pi)) ** (1.0 / 3.0)
    assert rg < 1.3 * rg_sphere  # compact parts: a random assignment gives ~3x, slabs ~2.8x


# ------------------------------------------------ library vs oracle (host C++)


@pytest.fixture(scope="module")
def H():
    import paper_1209_4506_amd.hartree as h

    return h


CASES = [(0, 1), (0, 4), (1, 1), (1, 5), (2, 2), (3, 7), (5, 8), (26, 4), (100, 3), (257, 19), (1000, 64), (4097, 33),
         (800, 1000)]


@pytest.mark.parametrize("natoms,nparts", CASES)
@pytest.mark.parametrize("weighted", [False, True])
def test_library_matches_oracle(H, natoms, nparts, weighted):
    x = cloud(natoms, 1000 + natoms + nparts)
    w = np.random.default_rng(natoms).uniform(0.05, 1.0, natoms) if weighted else None
    ref = op.decompose(x, nparts, w)
    got = H.atom_partition(x, nparts, w)
    for name, a, b in zip(("order", "part", "part_start"), got, ref):
        assert np.array_equal(a, b), name


@pytest.mark.parametrize("name,nparts", [("diamond16384", 19), ("diamond360", 8), ("diamond360", 16), ("diamond180", 5)])
def test_library_matches_oracle_diamond(H, name, nparts):
    p = getattr(inputs, name)()
    t = 1.0 + p.Z  # heavier atoms cost more: weights of Eq. (19), each time over the longest
    w = t / t.max()
    for weights in (None, w):
        ref = op.decompose(p.pos, nparts, weights)
        got = H.atom_partition(p.pos, nparts, weights)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)


def test_library_degenerate_lattice_valid(H):
    # a perfect simple-cubic lattice: the tensor is isotropic, every axis is a
    # principal axis, so only validity and the unit-weight counts are unique
    g = np.arange(6.0)
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    for nparts in (1, 2, 7, 19, 216, 300):
        order, part, start = H.atom_partition(x, nparts)
        check_valid(order, part, start, 216, nparts)
        assert np.diff(start).tolist() == counts_tree(216, nparts)
    same = np.zeros((10, 3))  # all atoms at one point: t = 0, ties by index
    order, part, start = H.atom_partition(same, 3)
    assert order.tolist() == list(range(10))
    assert np.diff(start).tolist() == counts_tree(10, 3)


def test_library_rejects_bad_arguments(H):
    x = cloud(10, 1)
    with pytest.raises(H.HartreeError):
        H.atom_partition(x, 0)
    bad = x.copy()
    bad[3, 1] = np.nan
    with pytest.raises(H.HartreeError):
        H.atom_partition(bad, 2)
    for w in (np.zeros(10), -np.ones(10), np.full(10, np.inf)):
        with pytest.raises(H.HartreeError):
            H.atom_partition(x, 2, w)
    assert H.LIB.hartree_atom_partition(-1, None, None, 1, None, None, None) == 1
