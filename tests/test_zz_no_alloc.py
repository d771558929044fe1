"""hartree_solve_noalloc (the entry point for callers that cannot allocate)
against hartree_solve, through the C ABI.

Two calls in a row on one GPU, the second on a smaller grid, share the
library's device scratch: each must match hartree_solve on its own input
(FP64: V rel-L2 <= 1e-12, E_H <= 1e-12; FP32: 5e-6 and 1e-6).  The plans used
with the no-allocation call have no workspace bound.
"""
import ctypes

import numpy as np
import pytest
import torch

from paper_1209_4506_amd import inputs

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a HIP device")]

TOL = {"fp64": (1e-12, 1e-12), "fp32": (5e-6, 1e-6)}
# (cell, dims) of the first call and of the smaller second one
CASES = [(np.diag([11.0, 12.0, 13.0]), (96, 90, 100)),
         (np.array([[9.0, 0.0, 0.0], [2.5, 8.0, 0.0], [-1.5, 2.0, 10.5]]), (36, 40, 30))]


def say(*a):
    print(*a, flush=True)


def vp(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_solve_noalloc_matches_solve(prec):
    import paper_1209_4506_amd.hartree as H

    dev = torch.device("cuda:0")
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    for call, (cell, dims) in enumerate(CASES):
        say("case no-alloc solve", prec, "call", call, "dims", dims)
        ref_plan = H.Plan(cell, dims, precision=prec, max_atoms=1)
        plan = H.Plan(cell, dims, precision=prec, max_atoms=1, bind=False)
        rho = torch.tensor(inputs.random_grid(dims, 40 + call), device=dev, dtype=ref_plan.dtype)
        V_ref, E_ref = ref_plan.solve(rho)
        V = torch.full(dims, float("nan"), device=dev, dtype=plan.dtype)
        E = torch.full((1,), float("nan"), device=dev, dtype=torch.float64)
        code = H.LIB.hartree_solve_noalloc(plan._h, vp(rho), vp(V), vp(E), stream)
        assert code == 0, H.LIB.hartree_last_error().decode()
        # V alone (no energy) on the same scratch
        V2 = torch.full(dims, float("nan"), device=dev, dtype=plan.dtype)
        code = H.LIB.hartree_solve_noalloc(plan._h, vp(rho), vp(V2), None, stream)
        assert code == 0, H.LIB.hartree_last_error().decode()
        torch.cuda.synchronize()
        ev = float(torch.linalg.vector_norm(V.double() - V_ref.double()) / torch.linalg.vector_norm(V_ref.double()))
        ee = abs(float(E[0]) - float(E_ref[0])) / abs(float(E_ref[0]))
        same = torch.equal(V, V_ref) and float(E[0]) == float(E_ref[0])
        say("  V rel-L2 %.2e  E_H rel %.2e  bit-identical %s" % (ev, ee, same))
        assert ev <= TOL[prec][0] and ee <= TOL[prec][1]
        assert torch.equal(V2, V)


def test_solve_noalloc_rejects_large_plans():
    import paper_1209_4506_amd.hartree as H

    say("case no-alloc solve, plan larger than the scratch")
    dims = (256, 256, 256)
    plan = H.Plan(np.eye(3) * 20.0, dims, precision="fp32", max_atoms=1, bind=False)
    rho = torch.zeros(dims, device="cuda", dtype=torch.float32)
    V = torch.empty_like(rho)
    code = H.LIB.hartree_solve_noalloc(plan._h, vp(rho), vp(V), None, None)
    assert code == 5  # HARTREE_ERR_WORKSPACE, before anything is enqueued
    assert "HARTREE_NOALLOC_BYTES" in H.LIB.hartree_last_error().decode()
