"""Thin Python binding of libhartree.so (the C ABI declared in include/hartree.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  PyTorch supplies device memory and the current stream.  Importing
this module loads the library and raises if it is missing -- there is no CPU
fallback.

Names follow the C ABI:

* ``Plan``                 -- hartree_plan_create[_batched] + workspace binding
* ``Plan.solve``           -- hartree_solve: V = P rho and E_H (Eq. (6), Eq. (7))
* ``Plan.energy``          -- hartree_energy
* ``Plan.backward``        -- hartree_backward: P (grad_v + grad_e dV rho)
* ``Plan.solve_backward``  -- hartree_solve_backward: both, as two concurrent
                              chains of passes
* ``Plan.splat``           -- hartree_splat: Gaussian atomic density
* ``Plan.splat_adjoint``   -- hartree_splat_adjoint: d/dR of sum grad_rho * rho
* ``atom_partition``       -- hartree_atom_partition: recursive bisection of
                              the atoms along inertia-tensor principal axes
* ``HartreeFn``            -- autograd function (pos -> V, E_H) whose backward
                              applies the symmetric P and the splat adjoint
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhartree.so")

FP64, FP32 = 0, 1
STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_DIMS", 3: "ERR_CELL", 4: "ERR_UNSUPPORTED", 5: "ERR_WORKSPACE", 6: "ERR_HIP"}
DEV_BAD_ATOM, DEV_SIGMA_RANGE, DEV_BIN_OVERFLOW = 0x1, 0x2, 0x4


class HartreeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS.get(code, str(code)), msg))
        self.code = code


class PlanOpts(ctypes.Structure):
    _fields_ = [("cutoff_sigmas", ctypes.c_double), ("max_sigma", ctypes.c_double),
                ("max_atoms", ctypes.c_int32), ("reserved", ctypes.c_int32 * 7)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libhartree.so is not built (run __graft_entry__.build() or "
                          "python -m paper_1209_4506_amd.build); there is no fallback path")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, d, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    P = ctypes.POINTER
    sig = {
        "hartree_plan_create": [P(vp), P(d), P(i32), i32, P(PlanOpts)],
        "hartree_plan_create_batched": [P(vp), i32, P(d), P(i32), i32, P(PlanOpts)],
        "hartree_plan_nprob": [vp, P(i32)],
        "hartree_plan_grid_offset": [vp, i32, P(i64)],
        "hartree_workspace_size": [vp, P(sz)],
        "hartree_bind_workspace": [vp, vp, sz],
        "hartree_solve": [vp, vp, vp, vp, vp],
        "hartree_energy": [vp, vp, vp, vp],
        "hartree_backward": [vp, vp, vp, vp, vp, vp],
        "hartree_solve_backward": [vp, vp, vp, vp, vp, vp, vp, vp],
        "hartree_splat": [vp, i32, vp, vp, vp, P(i32), vp, i32, vp],
        "hartree_splat_adjoint": [vp, i32, vp, vp, vp, P(i32), vp, vp, vp],
        "hartree_device_status": [vp, P(ctypes.c_uint32), vp],
        "hartree_atoms_bind": [vp, i32, vp, vp, vp, P(i32), P(ctypes.c_uint64), vp],
        "hartree_splat_bound": [vp, ctypes.c_uint64, vp, i32, vp],
        "hartree_splat_adjoint_bound": [vp, ctypes.c_uint64, vp, vp, vp],
        "hartree_profile_begin": [vp],
        "hartree_profile_end": [vp, P(d), P(i64)],
        "hartree_graph_begin": [vp, vp],
        "hartree_graph_end": [vp, vp],
        "hartree_graph_launch": [vp, vp],
        "hartree_plan_get_config": [vp, P(i32)],
        "hartree_plan_set_config": [vp, P(i32)],
        "hartree_plan_tune": [vp, vp, i32, vp],
        "hartree_atom_partition": [i32, P(d), P(d), i32, P(i32), P(i32), P(i32)],
        "hartree_atoms_pairs": [vp, P(i64), vp],
        "hartree_solve_noalloc": [vp, vp, vp, vp, vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.hartree_plan_destroy.argtypes = [vp]
    lib.hartree_plan_destroy.restype = None
    lib.hartree_last_error.argtypes = []
    lib.hartree_last_error.restype = ctypes.c_char_p
    return lib


LIB = _load()

# every symbol the header declares
EXPORTED = ["hartree_plan_create", "hartree_plan_create_batched", "hartree_plan_destroy", "hartree_plan_nprob",
            "hartree_plan_grid_offset", "hartree_workspace_size", "hartree_bind_workspace", "hartree_solve",
            "hartree_energy", "hartree_backward", "hartree_solve_backward", "hartree_splat", "hartree_splat_adjoint",
            "hartree_device_status", "hartree_atoms_bind", "hartree_splat_bound", "hartree_splat_adjoint_bound",
            "hartree_profile_begin", "hartree_profile_end", "hartree_graph_begin", "hartree_graph_end",
            "hartree_graph_launch", "hartree_plan_get_config", "hartree_plan_set_config", "hartree_plan_tune",
            "hartree_atom_partition", "hartree_atoms_pairs", "hartree_solve_noalloc", "hartree_last_error"]

# device scratch of hartree_solve_noalloc (HARTREE_NOALLOC_BYTES)
NOALLOC_BYTES = 64 * 1024 * 1024

# hartree_kernel_id order
KERNELS = ["r2c", "r2c_bwd", "fft_b", "fft_a", "fft_a_bwd", "fft_a_eonly", "fft_b_inv", "c2r", "finalize",
           "bin", "splat", "adjoint", "adjoint_final"]


def _check(code):
    if code != 0:
        raise HartreeError(code, LIB.hartree_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _opts(cutoff_sigmas=0.0, max_sigma=0.0, max_atoms=0):
    o = PlanOpts()
    o.cutoff_sigmas = float(cutoff_sigmas)
    o.max_sigma = float(max_sigma)
    o.max_atoms = int(max_atoms)
    return o


def atom_partition(pos, nparts, weights=None):
    """hartree_atom_partition on host arrays (Sec. 3.1).

    ``pos``: (natoms, 3) positions; ``weights``: (natoms,) positive or None.
    Returns ``(order, part, part_start)`` as int32 numpy arrays: atom indices
    grouped by part, the part of each atom, and the nparts + 1 offsets of the
    parts in ``order``.
    """
    if isinstance(pos, torch.Tensor):
        pos = pos.detach().cpu().numpy()
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    n = pos.shape[0]
    w = None
    if weights is not None:
        if isinstance(weights, torch.Tensor):
            weights = weights.detach().cpu().numpy()
        w = np.ascontiguousarray(weights, dtype=np.float64).reshape(-1)
        if w.shape[0] != n:
            raise HartreeError(1, "weights must have one entry per atom")
    order = np.empty(n, dtype=np.int32)
    part = np.empty(n, dtype=np.int32)
    start = np.empty(max(int(nparts), 0) + 1, dtype=np.int32)
    P = ctypes.POINTER
    dp = lambda a: a.ctypes.data_as(P(ctypes.c_double))  # noqa: E731
    ip = lambda a: a.ctypes.data_as(P(ctypes.c_int32))  # noqa: E731
    _check(LIB.hartree_atom_partition(n, dp(pos) if n else None, dp(w) if w is not None else None, int(nparts),
                                      ip(order), ip(part), ip(start)))
    return order, part, start


class Plan:
    """A solve plan for one cell (or a batch of cells) and its bound workspace.

    ``cells``: (3, 3) rows a, b, c in Bohr, or (nprob, 3, 3) for a batch.
    ``dims``: (Na, Nb, Nc), or (nprob, 3).  ``precision``: "fp32" or "fp64".
    Grid tensors are C-contiguous (Na, Nb, Nc) of the plan's dtype on the
    plan's device; a batched plan takes the grids flattened and concatenated.
    """

    def __init__(self, cells, dims, precision="fp32", device="cuda", cutoff_sigmas=0.0, max_sigma=0.0,
                 max_atoms=0, bind=True):
        cells = np.ascontiguousarray(cells, dtype=np.float64)
        dims = np.ascontiguousarray(dims, dtype=np.int32)
        self.batched = cells.ndim == 3
        if not self.batched:
            cells = cells.reshape(1, 3, 3)
            dims = dims.reshape(1, 3)
        self.nprob = cells.shape[0]
        self.cells = cells
        self.dims = [tuple(int(v) for v in r) for r in dims]
        self.precision = precision
        self.fp = FP64 if precision == "fp64" else FP32
        self.dtype = torch.float64 if self.fp == FP64 else torch.float32
        self.device = torch.device(device)
        h = ctypes.c_void_p()
        opts = _opts(cutoff_sigmas, max_sigma, max_atoms)
        cp = cells.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        dp = dims.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        if self.batched:
            _check(LIB.hartree_plan_create_batched(ctypes.byref(h), self.nprob, cp, dp, self.fp, ctypes.byref(opts)))
        else:
            _check(LIB.hartree_plan_create(ctypes.byref(h), cp, dp, self.fp, ctypes.byref(opts)))
        self._h = h
        off = ctypes.c_int64()
        self.offsets = []
        for p in range(self.nprob + 1):
            _check(LIB.hartree_plan_grid_offset(h, p, ctypes.byref(off)))
            self.offsets.append(int(off.value))
        self.volumes = np.abs(np.linalg.det(cells))
        self.workspace = None
        if bind:
            self.bind()

    # ------------------------------------------------------------ plumbing
    def workspace_size(self) -> int:
        n = ctypes.c_size_t()
        _check(LIB.hartree_workspace_size(self._h, ctypes.byref(n)))
        return int(n.value)

    def bind(self, workspace: torch.Tensor = None):
        need = self.workspace_size()
        if workspace is None:
            raw = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
            shift = (-raw.data_ptr()) % 256
            workspace = raw[shift:shift + need]
            self._ws_raw = raw
        _check(LIB.hartree_bind_workspace(self._h, ctypes.c_void_p(workspace.data_ptr()), need))
        self.workspace = workspace
        return self

    def __del__(self):
        if LIB is None:  # interpreter shutdown
            return
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            LIB.hartree_plan_destroy(h)
            self._h = None

    def grid_shape(self):
        return self.dims[0] if not self.batched else (self.offsets[-1],)

    def empty_grid(self):
        return torch.empty(self.grid_shape(), dtype=self.dtype, device=self.device)

    def _grid(self, t, name):
        if t is None:
            return None
        if t.dtype != self.dtype or t.device.type != "cuda" or not t.is_contiguous():
            raise TypeError("%s must be a contiguous %s CUDA tensor" % (name, self.dtype))
        if t.numel() != self.offsets[-1]:
            raise ValueError("%s has %d elements, the plan's grid has %d" % (name, t.numel(), self.offsets[-1]))
        return t

    # ------------------------------------------------------------ solve
    def solve(self, rho, v=None, e_h=None, stream=None):
        """V = P rho and E_H; returns (V, E_H) (E_H: float64 tensor of nprob)."""
        self._grid(rho, "rho")
        v = self.empty_grid() if v is None else self._grid(v, "v")
        e_h = torch.empty(self.nprob, dtype=torch.float64, device=self.device) if e_h is None else e_h
        _check(LIB.hartree_solve(self._h, _ptr(rho), _ptr(v), _ptr(e_h), stream or _stream(self.device)))
        return v, e_h

    def solve_noalloc(self, rho, v, e_h=None, stream=None):
        """hartree_solve_noalloc: V (and E_H into ``e_h`` if given) with the
        library's own device scratch; the plan needs no workspace.  ``v`` and
        ``e_h`` are preallocated by the caller."""
        self._grid(rho, "rho")
        self._grid(v, "v")
        _check(LIB.hartree_solve_noalloc(self._h, _ptr(rho), _ptr(v), _ptr(e_h), stream or _stream(self.device)))
        return v, e_h

    def potential(self, rho, v=None, stream=None):
        """V = P rho without the energy reduction."""
        self._grid(rho, "rho")
        v = self.empty_grid() if v is None else self._grid(v, "v")
        _check(LIB.hartree_solve(self._h, _ptr(rho), _ptr(v), None, stream or _stream(self.device)))
        return v

    def energy(self, rho, e_h=None, stream=None):
        self._grid(rho, "rho")
        e_h = torch.empty(self.nprob, dtype=torch.float64, device=self.device) if e_h is None else e_h
        _check(LIB.hartree_energy(self._h, _ptr(rho), _ptr(e_h), stream or _stream(self.device)))
        return e_h

    def backward(self, grad_v=None, grad_e=None, rho=None, out=None, stream=None):
        """grad_rho = P (grad_v + grad_e * dV * rho)."""
        self._grid(grad_v, "grad_v")
        self._grid(rho, "rho")
        if grad_e is not None:
            grad_e = grad_e.to(device=self.device, dtype=torch.float64).contiguous().reshape(-1)
            if grad_e.numel() != self.nprob:
                raise ValueError("grad_e needs one value per problem")
        out = self.empty_grid() if out is None else self._grid(out, "out")
        _check(LIB.hartree_backward(self._h, _ptr(grad_v), _ptr(grad_e), _ptr(rho), _ptr(out),
                                    stream or _stream(self.device)))
        return out

    def solve_backward(self, rho, grad_v=None, grad_e=None, v=None, e_h=None, out=None, stream=None):
        """solve and backward in one call (hartree_solve_backward): the
        backward needs rho and the upstream gradients, not V, so the two
        chains of passes run side by side when their spectra fit the cache;
        returns (V, E_H, grad_rho), identical to the two calls in order."""
        self._grid(rho, "rho")
        self._grid(grad_v, "grad_v")
        if grad_e is not None:
            grad_e = grad_e.to(device=self.device, dtype=torch.float64).contiguous().reshape(-1)
            if grad_e.numel() != self.nprob:
                raise ValueError("grad_e needs one value per problem")
        v = self.empty_grid() if v is None else self._grid(v, "v")
        e_h = torch.empty(self.nprob, dtype=torch.float64, device=self.device) if e_h is None else e_h
        out = self.empty_grid() if out is None else self._grid(out, "out")
        _check(LIB.hartree_solve_backward(self._h, _ptr(rho), _ptr(v), _ptr(e_h), _ptr(grad_v), _ptr(grad_e),
                                          _ptr(out), stream or _stream(self.device)))
        return v, e_h, out

    # ------------------------------------------------------------ atoms
    def _atoms(self, pos, Z, sigma, atom_counts):
        pos = pos.to(device=self.device, dtype=torch.float64).contiguous().reshape(-1, 3)
        Z = Z.to(device=self.device, dtype=torch.float64).contiguous().reshape(-1)
        sigma = sigma.to(device=self.device, dtype=torch.float64).contiguous().reshape(-1)
        n = pos.shape[0]
        if Z.numel() != n or sigma.numel() != n:
            raise ValueError("pos, Z and sigma disagree on the atom count")
        offs = None
        if self.batched:
            if atom_counts is None:
                raise ValueError("a batched plan needs atom_counts")
            c = np.concatenate([[0], np.cumsum(np.asarray(atom_counts, dtype=np.int64))]).astype(np.int32)
            offs = (ctypes.c_int32 * len(c))(*c.tolist())
        return pos, Z, sigma, n, offs

    def bind_atoms(self, pos, Z, sigma, atom_counts=None, stream=None):
        """Bin the atoms once for a splat and its adjoint; returns a token.
        The tensors passed here must stay alive and unchanged while it is used."""
        pos, Z, sigma, n, offs = self._atoms(pos, Z, sigma, atom_counts)
        token = ctypes.c_uint64()
        _check(LIB.hartree_atoms_bind(self._h, n, _ptr(pos), _ptr(Z), _ptr(sigma), offs, ctypes.byref(token),
                                      stream or _stream(self.device)))
        self._bound = (pos, Z, sigma, n)  # keep the converted arrays alive
        return int(token.value)

    def atoms_pairs(self, stream=None) -> int:
        """(atom, brick) pairs of the last binding (synchronous)."""
        n = ctypes.c_int64()
        _check(LIB.hartree_atoms_pairs(self._h, ctypes.byref(n), stream or _stream(self.device)))
        return int(n.value)

    def splat_bound(self, token, out=None, subtract_background=True, stream=None):
        out = self.empty_grid() if out is None else self._grid(out, "out")
        _check(LIB.hartree_splat_bound(self._h, ctypes.c_uint64(token), _ptr(out), 1 if subtract_background else 0,
                                       stream or _stream(self.device)))
        return out

    def splat_adjoint_bound(self, token, grad_rho, out=None, stream=None):
        self._grid(grad_rho, "grad_rho")
        n = self._bound[3]
        out = torch.empty((n, 3), dtype=torch.float64, device=self.device) if out is None else out
        _check(LIB.hartree_splat_adjoint_bound(self._h, ctypes.c_uint64(token), _ptr(grad_rho), _ptr(out),
                                               stream or _stream(self.device)))
        return out

    def splat(self, pos, Z, sigma, out=None, subtract_background=True, atom_counts=None, stream=None):
        pos, Z, sigma, n, offs = self._atoms(pos, Z, sigma, atom_counts)
        out = self.empty_grid() if out is None else self._grid(out, "out")
        _check(LIB.hartree_splat(self._h, n, _ptr(pos), _ptr(Z), _ptr(sigma), offs, _ptr(out),
                                 1 if subtract_background else 0, stream or _stream(self.device)))
        return out

    def splat_adjoint(self, pos, Z, sigma, grad_rho, out=None, atom_counts=None, stream=None):
        pos, Z, sigma, n, offs = self._atoms(pos, Z, sigma, atom_counts)
        self._grid(grad_rho, "grad_rho")
        out = torch.empty((n, 3), dtype=torch.float64, device=self.device) if out is None else out
        _check(LIB.hartree_splat_adjoint(self._h, n, _ptr(pos), _ptr(Z), _ptr(sigma), offs, _ptr(grad_rho),
                                         _ptr(out), stream or _stream(self.device)))
        return out

    def device_status(self) -> int:
        bits = ctypes.c_uint32()
        _check(LIB.hartree_device_status(self._h, ctypes.byref(bits), _stream(self.device)))
        return int(bits.value)

    def profile_begin(self):
        _check(LIB.hartree_profile_begin(self._h))

    def profile_end(self):
        """{kernel group: (total ms, launches)} since profile_begin (waits for the GPU)."""
        ms = (ctypes.c_double * len(KERNELS))()
        n = (ctypes.c_int64 * len(KERNELS))()
        _check(LIB.hartree_profile_end(self._h, ms, n))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNELS) if n[i]}

    def dv(self):
        return [float(self.volumes[p] / (self.offsets[p + 1] - self.offsets[p])) for p in range(self.nprob)]

    # ------------------------------------------------------------ pass shapes
    def get_config(self):
        """(nprob, 3, 3) int array: per problem and axis (a, b, c) the compiled
        radix plan entry (-1: run-time radix kernel), log2 pencils per tile and
        the LDS pitch pad of the strided axes."""
        buf = (ctypes.c_int32 * (9 * self.nprob))()
        _check(LIB.hartree_plan_get_config(self._h, buf))
        return np.array(buf[:], dtype=np.int32).reshape(self.nprob, 3, 3)

    def set_config(self, cfg):
        cfg = np.ascontiguousarray(cfg, dtype=np.int32).reshape(-1)
        if cfg.size != 9 * self.nprob:
            raise ValueError("config needs %d entries" % (9 * self.nprob))
        _check(LIB.hartree_plan_set_config(self._h, cfg.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))

    def cache_key(self):
        return "%s:%s" % (self.precision, ";".join("x".join(str(int(v)) for v in d) for d in self.dims))

    def tune(self, reps=5, cache=None):
        """Pick the fastest pass shapes on this device (see hartree_plan_tune).

        ``cache``: path of a JSON file keyed by precision and grid sizes; a hit
        applies the stored choice without timing, a miss tunes and stores it.
        Returns the applied config."""
        import json

        key = self.cache_key()
        table = {}
        if cache is not None and os.path.exists(cache):
            with open(cache) as fh:
                table = json.load(fh)
            if key in table:
                self.set_config(table[key])
                return self.get_config()
        scratch = self.empty_grid()
        _check(LIB.hartree_plan_tune(self._h, _ptr(scratch), int(reps), _stream(self.device)))
        del scratch
        cfg = self.get_config()
        if cache is not None:
            table[key] = cfg.reshape(-1).tolist()
            with open(cache, "w") as fh:
                json.dump(table, fh, indent=1, sort_keys=True)
        return cfg

    def capture(self, fn, stream=None):
        """Run ``fn()`` once eagerly, then record it into the plan's HIP graph.

        ``fn`` enqueues this plan's calls on the current stream and must write
        only into preallocated tensors (``out=`` arguments): nothing may be
        allocated while the stream is captured.  Capture runs on ``stream`` (a
        new side stream by default); replay with :meth:`replay`.
        """
        fn()
        s = stream or torch.cuda.Stream(self.device)
        s.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(s):
            h = ctypes.c_void_p(s.cuda_stream)
            _check(LIB.hartree_graph_begin(self._h, h))
            try:
                fn()
            finally:
                code = LIB.hartree_graph_end(self._h, h)
        _check(code)
        torch.cuda.current_stream(self.device).wait_stream(s)

    def replay(self, stream=None):
        """Launch the captured graph on the current stream (or ``stream``)."""
        _check(LIB.hartree_graph_launch(self._h, stream or _stream(self.device)))


class HartreeFn(torch.autograd.Function):
    """(pos) -> (V, E_H) through the splat and the Poisson solve.

    Backward: grad_rho = P (grad_V + grad_E dV rho), then the splat adjoint
    gives dL/dpos.  The real-space density from the forward is kept; its
    spectrum is recomputed by the backward transform rather than stored.
    """

    @staticmethod
    def forward(ctx, pos, Z, sigma, plan, atom_counts=None):
        token = plan.bind_atoms(pos.detach(), Z, sigma, atom_counts=atom_counts)
        rho = plan.splat_bound(token)
        V, E = plan.solve(rho)
        ctx.plan = plan
        ctx.atom_counts = atom_counts
        ctx.token = token
        ctx.save_for_backward(pos, Z, sigma, rho)
        return V, E

    @staticmethod
    def backward(ctx, gV, gE):
        pos, Z, sigma, rho = ctx.saved_tensors
        plan = ctx.plan
        gV = None if gV is None else gV.to(plan.dtype).contiguous()
        grho = plan.backward(grad_v=gV, grad_e=gE, rho=rho if gE is not None else None)
        try:  # the forward's binding, unless the plan has been rebound since
            gpos = plan.splat_adjoint_bound(ctx.token, grho)
        except HartreeError:
            gpos = plan.splat_adjoint(pos.detach(), Z, sigma, grho, atom_counts=ctx.atom_counts)
        return gpos.to(pos.dtype), None, None, None, None


def hartree(pos, Z, sigma, plan, atom_counts=None):
    """Differentiable (V, E_H) of Gaussian atoms at ``pos`` (see HartreeFn)."""
    return HartreeFn.apply(pos, Z, sigma, plan, atom_counts)
