#!/usr/bin/env python3
"""Hartree solves/sec on one MI355X: the 360^3 diamond workload, FP32 fwd+bwd.

One step (one "solve") is the whole hot path on one batch of synthetic input:
  bin        atoms into bricks (once, shared by splat and adjoint)
  splat      rho = sum of the Gaussians - Q/Omega
  solve      V = P rho, E_H                         (P1 .. P5 + E_H finalize)
  backward   grad_rho = P (c dV + 1 * dV * rho)     (loss L = E_H + <c, V> dV)
  adjoint    dL/dR for every atom
All inputs are resident in HBM before the timed region starts.

Prints one JSON line.  `value` is the rate of K steps of the 360^3 workload
replayed as one captured HIP graph each (the replayed outputs are checked bit
for bit against an eager step).  Beside it, per workload:
  eager       the same K steps launched kernel by kernel, every kernel group
              bracketed by HIP events (per-kernel times, the rooflines);
  replay_ms   min / median / mean of single replays, each timed with HIP
              events, over at least one second of replays;
  fp64_plain  the same step with an FP64 plan, eager (the comparison point);
and the same record for the 24-problem batched workload and the 1024^3
workload under `workloads`.  The CPU oracle is timed on a bounded sample of
the 360^3 workload.  --eager reports the eager rate as `value`.
"""
import argparse
import hashlib
import json
import math
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
WORKLOADS = ("diamond360", "batched24", "cubic1024")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the default pass shapes (skip hartree_plan_tune)")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON file of tuned pass shapes: applied when it holds a plan, else written after tuning")
    ap.add_argument("--eager", action="store_true",
                    help="time eager launches only (no HIP graph replay region; value is then the eager rate)")
    ap.add_argument("--cpu-atoms", type=int, default=4096, help="atoms in the CPU-oracle sample (all of them by default)")
    ap.add_argument("--workload", choices=WORKLOADS, default="diamond360",
                    help="the workload `value` is quoted on (the headline is diamond360)")
    ap.add_argument("--only", action="store_true",
                    help="run the --workload alone (no other workloads: for profiler runs)")
    ap.add_argument("--atom-order", choices=("given", "shuffled", "bisection"), default="given",
                    help="atom order handed to the library (diamond360): as generated (lattice order), a random "
                         "permutation, or the recursive-bisection order of hartree_atom_partition")
    ap.add_argument("--atom-parts", type=int, default=64, help="parts of the bisection order")
    ap.add_argument("--out", default=None, help="also write the JSON line to this file")
    ap.add_argument("--serial-chains", action="store_true",
                    help="replay the step with the solve and the backward in order (two calls) instead of "
                         "hartree_solve_backward, whose backward chain runs beside the solve's")
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
        # the loss weights c ~ N(0, 1) times dV, drawn on the device (a seeded
        # torch generator: a host draw of a 1024^3 grid takes tens of seconds)
        dvs = p.dv()
        self.gv = p.empty_grid()
        gen = torch.Generator(device=dev)
        for i, q in enumerate(probs):
            gen.manual_seed(1209 + i)
            part = self.gv.reshape(-1)[p.offsets[i]:p.offsets[i + 1]]
            part.normal_(generator=gen)
            part.mul_(dvs[i])
        self.ge = torch.ones(len(probs), dtype=torch.float64, device=dev)
        self.rho = p.empty_grid()
        self.V = p.empty_grid()
        self.E = torch.empty(len(probs), dtype=torch.float64, device=dev)
        self.grho = p.empty_grid()
        self.gpos = torch.empty((self.pos.shape[0], 3), dtype=torch.float64, device=dev)

    def __call__(self, fused=False):
        p = self.plan
        # binning shared by splat and adjoint
        token = p.bind_atoms(self.pos, self.Z, self.sig, atom_counts=self.counts)
        p.splat_bound(token, out=self.rho)
        if fused:
            # the backward chain (it needs rho and the loss weights, not V)
            # beside the solve's, on the plan's second stream and spectrum
            p.solve_backward(self.rho, grad_v=self.gv, grad_e=self.ge, v=self.V, e_h=self.E, out=self.grho)
        else:
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

    def timed_graph(self, steps, warmup, fused=True):
        """The step captured once as a HIP graph and replayed (with `fused`,
        the solve and backward as hartree_solve_backward's two concurrent
        chains); the replayed outputs are checked bit for bit against an
        eager step with the calls in order.  Returns (seconds for `steps`
        replays, bit-identical, per-replay milliseconds from HIP events over
        at least one second)."""
        torch = self.torch
        self()
        torch.cuda.synchronize()
        ref = self.outputs()
        self.plan.capture(lambda: self(fused=fused))
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
        # single replays bracketed by events on the replay stream (torch's current)
        n = max(steps, int(math.ceil(1.0 / max(dt / steps, 1e-6))))
        n = min(n, 20000)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * n)]
        for i in range(n):
            ev[2 * i].record()
            self.plan.replay()
            ev[2 * i + 1].record()
        torch.cuda.synchronize()
        per = sorted(ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(n))
        stats = {"min": per[0], "median": per[n // 2], "mean": sum(per) / n, "max": per[-1], "replays": n}
        return dt, same, stats


def window_points(probs, cutoff):
    """The method's splat work: sum over atoms of the product over the three
    axes of the grid points inside the atom's truncation window (at most the
    axis length), i.e. the (atom, grid point) pairs of the density sum."""
    import numpy as np

    total = 0
    for q in probs:
        L = np.diag(q.cell)
        w = np.ones(q.natoms)
        for x in range(3):
            n = q.dims[x]
            h = L[x] / n
            X = np.mod(q.pos[:, x], L[x])
            rc = cutoff * q.sigma
            lo = np.ceil((X - rc) / h)
            hi = np.floor((X + rc) / h)
            w *= np.minimum(hi - lo + 1, n)
        total += int(w.sum())
    return total


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


# The splat and adjoint count the method's own work: per (atom, window
# point) one multiply-add for the density (2 flops) and two for the adjoint
# (the factor and its displacement-weighted form, 4 flops).  The kernels
# execute more: whole 16 x 16 x 32 bricks per (atom, brick) pair, the adjoint
# as three 16-bit split products per FP32 product.
FLOPS_PER_POINT = {"splat": 2, "adjoint": 4}
EXEC_MULT = {"splat": 1, "adjoint": 3}


def roofline_of(name, probs, s, wpoints, pairs, avg_ms, traffic_file=None):
    """Roofline entry of one kernel group from its average launch time: the
    splat and adjoint against the FP32 matrix-core peak (method flops), the
    grid passes against HBM (algorithmic bytes)."""
    by = kernel_bytes(name, probs, s)
    if name in FLOPS_PER_POINT:
        fl = FLOPS_PER_POINT[name] * wpoints
        ach = fl / (avg_ms * 1e-3) / 1e12
        dense = FLOPS_PER_POINT[name] * BRICK_POINTS_F32 * pairs
        return {"bound": "mfma", "kernel": name, "achieved": ach, "peak": PEAK_MFMA_F32_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / PEAK_MFMA_F32_TFLOPS, "traffic": traffic_for(traffic_file, name),
                "method_flops_per_launch": fl, "window_points": wpoints,
                "brick_dense_flops_per_launch": dense, "atom_brick_pairs": pairs,
                "executed_mfma_flops_per_launch": EXEC_MULT[name] * dense,
                "bytes_per_launch": by, "hbm_gbs": by / (avg_ms * 1e-3) / 1e9, "avg_launch_us": 1000.0 * avg_ms}
    if by is None:
        return None
    ach = by / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": name, "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": ach / PEAK_HBM_GBS, "traffic": traffic_for(traffic_file, name), "bytes_per_launch": by,
            "avg_launch_us": 1000.0 * avg_ms}


def traffic_for(path, kernel):
    """Counter-measured HBM bytes per launch, if taken on the current sources."""
    if path is None:
        return None
    f = os.path.join(ROOT, "profiles", path)
    if not os.path.exists(f):
        return None
    with open(f) as fh:
        t = json.load(fh)
    if t.get("source_hash") != source_hash():
        return None
    return t.get("kernels", {}).get("fp32", {}).get(kernel)


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


def describe(name, probs):
    if name == "diamond360":
        return ("diamond360: 8x8x8 diamond supercell, a = 53.93 Bohr, 4096 Gaussian atoms (Z = 4, sigma = 0.8 Bohr, "
                "N(0, 0.05) displacements, seed 1211), 360^3 grid, FP32 transforms with FP64 E_H and force "
                "reductions, splat + solve + backward + adjoint per step"), {"grid": list(probs[0].dims),
                                                                            "atoms": probs[0].natoms}
    if name == "cubic1024":
        return ("cubic1024: cubic cell a = 150 Bohr, 32768 uniform Gaussian atoms (Z = 4, sigma = 0.8 Bohr, seed "
                "1213), 1024^3 grid, FP32 transforms with FP64 E_H and force reductions, splat + solve + backward + "
                "adjoint per step"), {"grid": list(probs[0].dims), "atoms": probs[0].natoms}
    return ("batched24: 24 orthorhombic cells (edges U[8, 40] Bohr, each grid dimension from {48, 60, 72, 90, 120, "
            "150, 180, 240}, 16-512 atoms with Z in {1, 4, 6} and sigma U[0.6, 1.0]) in one batched plan, FP32 "
            "transforms with FP64 reductions, splat + solve + backward + adjoint of all 24 per step; solves count "
            "problems"), {"problems": len(probs), "points": int(sum(q.npoints for q in probs)),
                          "atoms": int(sum(q.natoms for q in probs))}


def problems(name, inputs, args, H):
    if name == "diamond360":
        prob, part_ms = reorder_atoms(inputs.diamond360(), args.atom_order, args.atom_parts, H)
        return [prob], part_ms
    if name == "cubic1024":
        return [inputs.cubic1024()], None
    return inputs.batched24(), None


def run_workload(name, args, torch, H, inputs, steps, warmup, fp64_steps):
    """One workload's record: graph-replayed rate, eager per-kernel times and
    rooflines, single-replay statistics, and the FP64 plain step."""
    probs, part_ms = problems(name, inputs, args, H)
    nprob = len(probs)
    desc, wconf = describe(name, probs)
    step = Step(probs, "fp32", torch, H, inputs, tune=not args.no_tune, cache=args.tune_cache)
    assert step.plan.device_status() == 0
    dt_eager, prof = step.timed(steps, warmup, profile=True)
    assert step.plan.device_status() == 0, "device status bits set"
    eager = {"value": nprob * steps / dt_eager, "unit": "solves/s", "ms_per_step": 1000.0 * dt_eager / steps}
    stats = None
    if args.eager:
        dt = dt_eager
        mode = "eager launches, per-kernel HIP events"
    else:
        dt, same, stats = step.timed_graph(steps, warmup, fused=not args.serial_chains)
        assert same, "graph replay differs from the eager step"
        assert step.plan.device_status() == 0, "device status bits set"
        mode = ("HIP graph replay of the whole step" +
                (" (solve, then backward)" if args.serial_chains else
                 " (hartree_solve_backward: the solve's and the backward's chains side by side when their spectra fit the cache)") +
                "; outputs bit-identical to the eager step with the calls in order; per-kernel times from "
                "that eager step")
    ms = 1000.0 * dt / steps
    s = 4
    n = sum(q.npoints for q in probs)
    model_bytes = 23 * s * n
    pairs = step.plan.atoms_pairs()
    wpts = window_points(probs, 6.0)
    tfile = "traffic_%s.json" % name
    rooflines = {k: roofline_of(k, probs, s, wpts, pairs, v[0] / v[1], tfile) for k, v in prof.items()}
    rooflines = {k: v for k, v in rooflines.items() if v is not None}
    dom = max(rooflines, key=lambda k: prof[k][0])
    per_kernel = {k: {"avg_us": round(1000.0 * v[0] / v[1], 2), "launches": v[1],
                      "share": round(v[0] / sum(x[0] for x in prof.values()), 4)} for k, v in prof.items()}
    rec = {
        "value": nprob * steps / dt,
        "unit": "solves/s",
        "ms_per_step": ms,
        "steps": steps,
        "timing": mode,
        "config": dict({"workload": desc}, **wconf, precision="fp32"),
        "hbm_gbs_model": model_bytes / (ms * 1e-3) / 1e9,
        "hbm_frac_model": model_bytes / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
        "roofline": rooflines[dom],
        "kernel_rooflines": {k: {"bound": v["bound"], "achieved": round(v["achieved"], 2), "unit": v["unit"],
                                 "frac": round(v["frac"], 4)} for k, v in rooflines.items()},
        "kernels": per_kernel,
        "pass_config": step.config.reshape(-1).tolist() if nprob == 1 else "per problem (see tune cache)",
        "eager": eager,
    }
    if stats is not None:
        rec["replay_ms"] = {k: (round(v, 5) if isinstance(v, float) else v) for k, v in stats.items()}
        rec["value_at_median_replay"] = nprob / (stats["median"] * 1e-3)
    if part_ms is not None:
        rec["atom_order"] = {"mode": args.atom_order,
                             "parts": args.atom_parts if args.atom_order == "bisection" else None,
                             "host_ms": part_ms}
    del step
    torch.cuda.empty_cache()
    if not args.no_fp64:
        step64 = Step(probs, "fp64", torch, H, inputs, tune=not args.no_tune, cache=args.tune_cache)
        dt64, prof64 = step64.timed(fp64_steps, 2, profile=True)
        assert step64.plan.device_status() == 0, "device status bits set"
        rec["fp64_plain"] = {"value": nprob * fp64_steps / dt64, "unit": "solves/s",
                             "ms_per_step": 1000.0 * dt64 / fp64_steps, "steps": fp64_steps,
                             "hbm_gbs_model": 23 * 8 * n / (dt64 / fp64_steps) / 1e9,
                             "kernels": {k: round(1000.0 * v[0] / v[1], 2) for k, v in prof64.items()}}
        rec["speedup_vs_fp64_plain"] = rec["value"] / rec["fp64_plain"]["value"]
        del step64
        torch.cuda.empty_cache()
    return rec, probs


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

    head, probs = run_workload(args.workload, args, torch, H, inputs, args.steps, args.warmup,
                               max(3, args.steps // 4))
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": head["config"],
        "roofline": head["roofline"],
    }
    for k in ("hbm_gbs_model", "hbm_frac_model", "replay_ms", "value_at_median_replay", "timing", "eager",
              "kernel_rooflines", "kernels", "pass_config", "fp64_plain", "speedup_vs_fp64_plain", "atom_order"):
        if k in head:
            out[k] = head[k]
    out["source_hash"] = source_hash()
    if not args.only:
        others = {}
        for name in WORKLOADS:
            if name == args.workload:
                continue
            # the 1024^3 step takes tens of milliseconds: fewer steps keep the run short
            k = args.steps if name != "cubic1024" else max(5, args.steps // 5)
            rec, _ = run_workload(name, args, torch, H, inputs, k, min(args.warmup, 3), 3)
            others[name] = rec
        out["workloads"] = others
    if not args.no_cpu_baseline and args.workload == "diamond360":
        out["cpu_baseline"] = cpu_baseline(probs[0], args.cpu_atoms, inputs)
    line = json.dumps(out)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(line + "\n")


if __name__ == "__main__":
    main()
