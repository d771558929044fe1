"""One-launch replay of a whole fwd+bwd step (hartree_graph_begin / end / launch).

Every replay is checked bit for bit against the same sequence run eagerly on
the same plan (the kernels and their reduction orders are identical), with
the program's own eager work and synchronisations between replays, and after
the atoms move in place (the binning is inside the captured sequence).
"""
import numpy as np
import pytest
import torch

from paper_1209_4506_amd import inputs

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a HIP device")]


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def H():
    import paper_1209_4506_amd.hartree as h

    return h


class Step:
    """Preallocated buffers and the calls of one step on a (batched) plan."""

    def __init__(self, H, probs, prec):
        dev = torch.device("cuda")
        cells = np.stack([q.cell for q in probs])
        dims = np.array([q.dims for q in probs])
        self.counts = [q.natoms for q in probs]
        self.plan = H.Plan(cells if len(probs) > 1 else cells[0], dims if len(probs) > 1 else dims[0],
                           precision=prec, max_atoms=int(sum(self.counts)))
        p = self.plan
        self.pos = torch.tensor(np.concatenate([q.pos for q in probs]), device=dev)
        self.Z = torch.tensor(np.concatenate([q.Z for q in probs]), device=dev)
        self.sig = torch.tensor(np.concatenate([q.sigma for q in probs]), device=dev)
        c = np.concatenate([inputs.random_grid(q.dims, 40 + i).reshape(-1) for i, q in enumerate(probs)])
        dvs = np.repeat(p.dv(), [q.npoints for q in probs])
        self.gv = torch.tensor(c * dvs, device=dev).to(p.dtype).reshape(p.grid_shape()).contiguous()
        self.ge = torch.ones(p.nprob, dtype=torch.float64, device=dev)
        self.rho = p.empty_grid()
        self.V = p.empty_grid()
        self.E = torch.empty(p.nprob, dtype=torch.float64, device=dev)
        self.grho = p.empty_grid()
        self.gpos = torch.empty((self.pos.shape[0], 3), dtype=torch.float64, device=dev)
        self.token = None

    def run(self, rebind=True):
        p = self.plan
        counts = self.counts if p.batched else None
        if rebind:
            self.token = p.bind_atoms(self.pos, self.Z, self.sig, atom_counts=counts)
        p.splat_bound(self.token, out=self.rho)
        p.solve(self.rho, v=self.V, e_h=self.E)
        p.backward(grad_v=self.gv, grad_e=self.ge, rho=self.rho, out=self.grho)
        p.splat_adjoint_bound(self.token, self.grho, out=self.gpos)

    def outputs(self):
        return [t.clone() for t in (self.rho, self.V, self.E, self.grho, self.gpos)]

    def scribble(self):
        """Eager work between replays: overwrite every output."""
        for t in (self.rho, self.V, self.grho):
            t.fill_(123.0)
        self.E.fill_(-1.0)
        self.gpos.fill_(float("nan"))


def assert_same(got, ref, what):
    names = ["rho", "V", "E_H", "grad_rho", "grad_pos"]
    for n, g, r in zip(names, got, ref):
        assert torch.equal(g, r), "%s: %s differs from the eager run" % (what, n)


def check_graph(step, rebind):
    step.run(rebind=True)
    torch.cuda.synchronize()
    assert step.plan.device_status() == 0
    ref = step.outputs()
    step.plan.capture(lambda: step.run(rebind=rebind))
    torch.cuda.synchronize()
    assert_same(step.outputs(), ref, "capture run")
    for rep in range(3):
        step.scribble()
        torch.cuda.synchronize()
        step.plan.replay()
        torch.cuda.synchronize()
        assert_same(step.outputs(), ref, "replay %d" % rep)
    return ref


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_graph_batched_replays_and_moved_atoms(H, prec):
    probs = [inputs.small_problem((30, 36, 40), 25, seed=61, L=(8.0, 8.5, 9.0)),
             inputs.small_problem((21, 16, 27), 12, seed=62, L=(7.0, 9.0, 8.0)),
             inputs.small_problem((48, 20, 35), 40, seed=63, L=(12.0, 6.0, 10.0))]
    say("case graph batched", prec, [q.dims for q in probs])
    step = Step(H, probs, prec)
    check_graph(step, rebind=True)
    # move the atoms in place: the replay re-bins them
    step.pos.add_(torch.tensor(np.random.default_rng(5).normal(0.0, 0.3, tuple(step.pos.shape)), device="cuda"))
    torch.cuda.synchronize()
    step.plan.replay()
    torch.cuda.synchronize()
    got = step.outputs()
    step.run(rebind=True)
    torch.cuda.synchronize()
    assert_same(got, step.outputs(), "replay after moving the atoms")
    assert step.plan.device_status() == 0


def test_graph_single_plan_bound_outside(H):
    p = inputs.cubic32()
    say("case graph cubic32 fp32, binding outside the graph")
    step = Step(H, [p], "fp32")
    check_graph(step, rebind=False)


def test_graph_errors(H):
    say("case graph argument errors")
    p = inputs.cubic32()
    plan = H.Plan(p.cell, p.dims, precision="fp32", max_atoms=p.natoms)
    with pytest.raises(H.HartreeError):
        plan.replay()  # nothing captured yet
    assert H.LIB.hartree_graph_begin(plan._h, None) != 0  # the default stream cannot be captured
    s = torch.cuda.Stream()
    import ctypes

    assert H.LIB.hartree_graph_end(plan._h, ctypes.c_void_p(s.cuda_stream)) != 0  # no capture open
