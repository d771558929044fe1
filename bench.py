#!/usr/bin/env python3
"""Hartree solves/sec on one MI355X: the 360^3 diamond workload, FP32 fwd+bwd.

One step (one "solve") is the whole hot path on one batch of synthetic input:
  bin        atoms into bricks (once, shared by splat and adjoint)
  splat      rho = sum of 4096 Gaussians (Z = 4, sigma = 0.8 Bohr) - Q/Omega
  solve      V = P rho, E_H                         (P1 .. P5 + E_H finalize)
  backward   grad_rho = P (c dV + 1 * dV * rho)     (loss L = E_H + <c, V> dV)
  adjoint    dL/dR for every atom
All inputs are resident in HBM before the timed region starts.

Prints one JSON line.  `value` is the rate of K steps replayed as one
captured HIP graph each (the replayed outputs are checked bit for bit against
an eager step); `eager` is the rate of the same K steps launched kernel by
kernel with every kernel group bracketed by HIP events, which give the
per-kernel timings and the roofline of the dominant kernel.  Also: the same
step with an FP64 plan, eager (the "plain FP64" comparison), and the CPU
oracle timed on a bounded sample of the same workload.  --eager skips the
graph region and reports the eager rate as `value`.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_MFMA_F32_TFLOPS = 157.3  # MI355X dense FP32 matrix-core peak
PEAK_MFMA_F16_TFLOPS = 2500.0  # MI355X dense FP16 matrix-core peak
BRICK_POINTS_F32 = 16 * 16 * 32  # points of one FP32 splat brick
METRIC = "Hartree solves/sec & HBM GB/s, 360^3 FP32 fwd+bwd vs FP64 plain"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the default pass shapes (skip hartree_plan_tune)")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON file of tuned pass shapes: applied when it holds this plan, else written after tuning")
    ap.add_argument("--eager", action="store_true",
                    help="time eager launches only (no HIP graph replay region; value is then the eager rate)")
    ap.add_argument("--cpu-atoms", type=int, default=4096, help="atoms in the CPU-oracle sample (all of them by default)")
    ap.add_argument("--workload", choices=("diamond360", "batched24"), default="diamond360",
                    help="the headline 360^3 problem, or 24 uneven orthorhombic problems in one batched plan "
                         "(solves/s then counts problems)")
    ap.add_argument("--atom-order", choices=("given", "shuffled", "bisection"), default="given",
                    help="atom order handed to the library: as generated (lattice order), a random "
                         "permutation, or the recursive-bisection order of hartree_atom_partition")
    ap.add_argument("--atom-parts", type=int, default=64, help="parts of the bisection order")
    ap.add_argument("--out", default=None, help="also write the JSON line to this file")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (to calibrate HBM byte counters)")
    return ap.parse_args()


def copy_calibration(torch):
    """Three device-to-device copies of 512 MiB each: the reference a byte
    counter (FETCH_SIZE, WRITE_SIZE) is scaled by."""
    n = 128 * 1024 * 1024
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": 4 * n, "copy_calibration_bytes_written": 4 * n,
                      "launches": 3}), flush=True)


def source_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1209_4506_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def reorder_atoms(prob, mode, nparts, H):
    """The same atoms in another order; returns (problem, host ms of the partition)."""
    import dataclasses

    import numpy as np

    if mode == "given":
        return prob, None
    t0 = time.perf_counter()
    if mode == "shuffled":
        perm = np.random.default_rng(prob.seed + 7).permutation(prob.natoms)
    else:
        perm = H.atom_partition(prob.pos, nparts)[0]
    ms = 1000.0 * (time.perf_counter() - t0)
    return dataclasses.replace(prob, pos=prob.pos[perm].copy(), Z=prob.Z[perm].copy(),
                               sigma=prob.sigma[perm].copy()), ms


class Step:
    """Preallocated buffers and the four C-ABI calls of one fwd+bwd solve of
    one problem, or of a batch of problems on one batched plan."""

    def __init__(self, probs, precision, torch, H, inputs, tune=True, cache=None):
        import numpy as np

        self.torch = torch
        dev = torch.device("cuda:0")
        batched = len(probs) > 1
        cells = np.stack([q.cell for q in probs])
        dims = np.array([q.dims for q in probs])
        self.counts = [q.natoms for q in probs] if batched else None
        self.plan = H.Plan(cells if batched else cells[0], dims if batched else dims[0], precision=precision,
                           device=dev, max_atoms=sum(q.natoms for q in probs))
        p = self.plan
        self.config = p.tune(reps=5, cache=cache) if tune else p.get_config()
        self.pos = torch.tensor(np.concatenate([q.pos for q in probs]), device=dev)
        self.Z = torch.tensor(np.concatenate([q.Z for q in probs]), device=dev)
        self.sig = torch.tensor(np.concatenate([q.sigma for q in probs]), device=dev)
        dvs = p.dv()
        c = np.concatenate([inputs.random_grid(q.dims, 1209 + i).reshape(-1) * dvs[i] for i, q in enumerate(probs)])
        self.gv = torch.tensor(c, device=dev).to(p.dtype).reshape(p.empty_grid().shape).contiguous()
        self.ge = torch.ones(len(probs), dtype=torch.float64, device=dev)
        self.rho = p.empty_grid()
        self.V = p.empty_grid()
        self.E = torch.empty(len(probs), dtype=torch.float64, device=dev)
        self.grho = p.empty_grid()
        self.gpos = torch.empty((self.pos.shape[0], 3), dtype=torch.float64, device=dev)

    def __call__(self):
        p = self.plan
        # binning shared by splat and adjoint
        token = p.bind_atoms(self.pos, self.Z, self.sig, atom_counts=self.counts)
        p.splat_bound(token, out=self.rho)
        p.solve(self.rho, v=self.V, e_h=self.E)
        p.backward(grad_v=self.gv, grad_e=self.ge, rho=self.rho, out=self.grho)
        p.splat_adjoint_bound(token, self.grho, out=self.gpos)

    def timed(self, steps, warmup, profile=False):
        torch = self.torch
        for _ in range(warmup):
            self()
        torch.cuda.synchronize()
        if profile:
            self.plan.profile_begin()
        t0 = time.perf_counter()
        for _ in range(steps):
            self()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = self.plan.profile_end() if profile else None
        return (t1 - t0), prof

    def outputs(self):
        return [t.clone() for t in (self.rho, self.V, self.E, self.grho, self.gpos)]

    def timed_graph(self, steps, warmup):
        """The same step captured once as a HIP graph and replayed; the
        replayed outputs are checked bit for bit against an eager step."""
        torch = self.torch
        self()
        torch.cuda.synchronize()
        ref = self.outputs()
        self.plan.capture(self)
        for _ in range(warmup):
            self.plan.replay()
        torch.cuda.synchronize()
        for t in (self.rho, self.V, self.grho, self.gpos, self.E):
            t.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            self.plan.replay()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        same = all(torch.equal(a, b) for a, b in zip(self.outputs(), ref))
        return dt, same


def kernel_bytes(name, probs, s):
    """Algorithmic HBM bytes of one launch of a kernel group over the
    problems of the plan (s = bytes per real)."""
    total = 0
    for prob in probs:
        na, nb, nc = prob.dims
        n = na * nb * nc
        spec = na * nb * (nc // 2 + 1) * 2 * s  # half spectrum, complex
        b = {
            "r2c": n * s + spec,
            "r2c_bwd": 2 * n * s + spec,
            "fft_b": 2 * spec,
            "fft_b_inv": 2 * spec,
            "fft_a": 2 * spec,
            "fft_a_bwd": 2 * spec,
            "c2r": spec + n * s,
            "splat": n * s,
            "adjoint": n * s,
        }.get(name)
        if b is None:
            return None
        total += b
    return total


def kernel_flops(name, pairs):
    """Algorithmic matrix-core flops of one launch of the splat or adjoint:
    per (atom, brick) pair one multiply-add per brick point (splat: the
    density; adjoint: two, the factor and its displacement-weighted form)."""
    per = {"splat": 2, "adjoint": 4}.get(name)
    return None if per is None else per * BRICK_POINTS_F32 * pairs


# the adjoint forms each FP32 product from three 16-bit products of split
# operands: its matrix cores execute three times the algorithmic flops, at
# the FP16 peak
MFMA_EXEC = {"splat": (1, PEAK_MFMA_F32_TFLOPS), "adjoint": (3, PEAK_MFMA_F16_TFLOPS)}


def roofline_of(name, probs, s, pairs, avg_ms, precision="fp32"):
    """Roofline entry of one kernel group from its average launch time: the
    matrix-core kernels (splat, adjoint) against the FP32 MFMA peak, the
    grid passes against HBM."""
    fl = kernel_flops(name, pairs)
    by = kernel_bytes(name, probs, s)
    if fl is not None:
        mult, peak = MFMA_EXEC[name]
        alg = fl / (avg_ms * 1e-3) / 1e12
        ach = mult * alg
        return {"bound": "mfma", "kernel": name, "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                "frac": ach / peak, "traffic": traffic_for(name, precision),
                "flops_per_launch": mult * fl, "algorithmic_flops_per_launch": fl,
                "fp32_equivalent_tflops": alg, "fp32_equivalent_frac": alg / PEAK_MFMA_F32_TFLOPS,
                "atom_brick_pairs": pairs, "bytes_per_launch": by,
                "hbm_gbs": by / (avg_ms * 1e-3) / 1e9, "avg_launch_us": 1000.0 * avg_ms}
    if by is None:
        return None
    ach = by / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": name, "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": ach / PEAK_HBM_GBS, "traffic": traffic_for(name, precision), "bytes_per_launch": by,
            "avg_launch_us": 1000.0 * avg_ms}


def traffic_for(kernel, precision):
    """Counter-measured HBM bytes per launch, if taken on the current sources."""
    f = os.path.join(ROOT, "profiles", "traffic_diamond360.json")
    if not os.path.exists(f):
        return None
    with open(f) as fh:
        t = json.load(fh)
    if t.get("source_hash") != source_hash():
        return None
    return t.get("kernels", {}).get(precision, {}).get(kernel)


def cpu_baseline(prob, natoms_sample, inputs):
    """The oracle on a bounded sample: the full-grid transforms of one step
    (forward solve and backward) plus splat and adjoint for a subset of the
    atoms, scaled to the whole atom count."""
    import numpy as np

    import oracle

    cell9 = prob.cell.reshape(9)
    k = min(natoms_sample, prob.natoms)
    sel = np.arange(k)
    t0 = time.perf_counter()
    rho = oracle.splat(cell9, prob.dims, prob.pos[sel], prob.Z[sel], prob.sigma[sel])
    t1 = time.perf_counter()
    V, _, E, _ = oracle.poisson(cell9, rho)
    dv = abs(np.linalg.det(prob.cell)) / prob.npoints
    c = inputs.random_grid(prob.dims, 1209)
    g = oracle.backward(cell9, rho, grad_v=c * dv, grad_e=1.0)
    t2 = time.perf_counter()
    oracle.splat_adjoint(cell9, prob.pos[sel], prob.Z[sel], prob.sigma[sel], g)
    t3 = time.perf_counter()
    scale = prob.natoms / k
    t_step = (t2 - t1) + scale * ((t1 - t0) + (t3 - t2))
    return {
        "value": 1.0 / t_step,
        "unit": "solves/s",
        "cores": oracle.max_threads(),
        "kind": "oracle",
        "sample": "one step on the full %dx%dx%d grid (forward solve + backward transforms, %.1f s) with the "
                  "splat and adjoint of %d of %d atoms (%.1f s) scaled x%.0f; measured %.1f s" % (
                      *prob.dims, t2 - t1, k, prob.natoms, (t1 - t0) + (t3 - t2), scale, t3 - t0),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (the sharded "
              "design is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    if args.copy_calibration:
        copy_calibration(torch)
        return

    import paper_1209_4506_amd.hartree as H
    from paper_1209_4506_amd import inputs

    if args.workload == "diamond360":
        prob, part_ms = reorder_atoms(inputs.diamond360(), args.atom_order, args.atom_parts, H)
        probs = [prob]
        workload = ("diamond360: 8x8x8 diamond supercell, a = 53.93 Bohr, 4096 Gaussian atoms (Z = 4, sigma = 0.8 "
                    "Bohr, N(0, 0.05) displacements, seed 1211), 360^3 grid, FP32 transforms with FP64 E_H and "
                    "force reductions, splat + solve + backward + adjoint per step")
        wconf = {"grid": list(prob.dims), "atoms": prob.natoms}
    else:
        probs, part_ms = inputs.batched24(), None
        workload = ("batched24: 24 orthorhombic cells (edges U[8, 40] Bohr, each grid dimension from {48, 60, 72, "
                    "90, 120, 150, 180, 240}, 16-512 atoms with Z in {1, 4, 6} and sigma U[0.6, 1.0]) in one "
                    "batched plan, FP32 transforms with FP64 reductions, splat + solve + backward + adjoint of all "
                    "24 per step; solves count problems")
        wconf = {"problems": len(probs), "points": int(sum(q.npoints for q in probs)),
                 "atoms": int(sum(q.natoms for q in probs))}
    nprob = len(probs)
    step = Step(probs, "fp32", torch, H, inputs, tune=not args.no_tune, cache=args.tune_cache)
    assert step.plan.device_status() == 0
    # eager region: every kernel group bracketed by HIP events (the roofline)
    dt_eager, prof = step.timed(args.steps, args.warmup, profile=True)
    assert step.plan.device_status() == 0, "device status bits set"
    eager = {"value": nprob * args.steps / dt_eager, "unit": "solves/s", "ms_per_step": 1000.0 * dt_eager / args.steps}
    if args.eager:
        dt = dt_eager
        mode = "eager launches, per-kernel HIP events"
    else:
        # the headline region: the same step replayed as one HIP graph
        dt, same = step.timed_graph(args.steps, args.warmup)
        assert same, "graph replay differs from the eager step"
        assert step.plan.device_status() == 0, "device status bits set"
        mode = "HIP graph replay of the whole step (outputs bit-identical to the eager step)"
    ms = 1000.0 * dt / args.steps
    s = 4
    n = sum(q.npoints for q in probs)
    model_bytes = 23 * s * n
    # dominant kernel group by time
    groups = {k: v for k, v in prof.items()}
    pairs = step.plan.atoms_pairs()
    rooflines = {k: roofline_of(k, probs, s, pairs, v[0] / v[1]) for k, v in groups.items()}
    rooflines = {k: v for k, v in rooflines.items() if v is not None}
    dom = max(rooflines, key=lambda k: groups[k][0])
    per_kernel = {k: {"avg_us": round(1000.0 * v[0] / v[1], 2), "launches": v[1],
                      "share": round(v[0] / sum(x[0] for x in groups.values()), 4)} for k, v in groups.items()}
    out = {
        "metric": METRIC,
        "value": nprob * args.steps / dt,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": dict({"workload": workload}, **wconf, precision="fp32"),
        "hbm_gbs_model": model_bytes / (ms * 1e-3) / 1e9,
        "roofline": rooflines[dom],
        "kernel_rooflines": {k: {"bound": v["bound"], "achieved": round(v["achieved"], 2), "unit": v["unit"],
                                 "frac": round(v["frac"], 4)} for k, v in rooflines.items()},
        "kernels": per_kernel,
        "pass_config": step.config.reshape(-1).tolist(),
        "source_hash": source_hash(),
    }
    out["timing"] = mode
    out["eager"] = eager
    if args.atom_order != "given":
        out["atom_order"] = {"mode": args.atom_order, "parts": args.atom_parts if args.atom_order == "bisection" else None,
                             "host_ms": part_ms}
    if not args.no_fp64:
        del step
        torch.cuda.empty_cache()
        step64 = Step(probs, "fp64", torch, H, inputs, tune=not args.no_tune, cache=args.tune_cache)
        k64 = max(3, args.steps // 4)
        dt64, prof64 = step64.timed(k64, 2, profile=True)
        out["fp64_plain"] = {"value": nprob * k64 / dt64, "unit": "solves/s", "ms_per_step": 1000.0 * dt64 / k64,
                             "steps": k64, "hbm_gbs_model": 23 * 8 * n / (dt64 / k64) / 1e9,
                             "kernels": {k: round(1000.0 * v[0] / v[1], 2) for k, v in prof64.items()}}
        out["speedup_vs_fp64_plain"] = out["value"] / out["fp64_plain"]["value"]
        del step64
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline and args.workload == "diamond360":
        out["cpu_baseline"] = cpu_baseline(probs[0], args.cpu_atoms, inputs)
    line = json.dumps(out)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(line + "\n")


if __name__ == "__main__":
    main()
