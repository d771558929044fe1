/*
 * hartree.h -- C ABI of the MI355X periodic Hartree (FFT-Poisson) library.
 *
 * The library computes, on one GPU, the Hartree potential of a density given
 * on a periodic real-space grid, its energy, the gradient of a loss through
 * both, the Gaussian atomic density that feeds the solve, and that density's
 * adjoint (Hartree forces on atoms).  Paper: Duy & Ozaki, "A three-dimensional
 * domain decomposition method for large-scale DFT electronic structure
 * calculations" (arXiv:1209.4506).
 *
 * Units are Hartree atomic units throughout: Bohr, Hartree, electron charge.
 *
 * Grid convention (Sec. 3.2.2, structure B in "abc" order): the cell rows are
 * the axes a, b, c; the grid has Na x Nb x Nc points at
 * r_ijk = (i/Na) a + (j/Nb) b + (k/Nc) c, stored row-major as
 * [Na][Nb][Nc] with the c index fastest.  Every grid array passed to the
 * library uses this layout.
 *
 * Precision: a plan is FP64 or FP32.  Every grid array passed to a plan holds
 * elements of the plan's precision (double or float).  Energies, atom
 * positions, charges, widths and gradients with respect to positions are
 * always double.
 *
 * Memory ownership: the caller owns all device memory.  The plan owns only
 * host metadata; its device workspace (twiddle tables, the half spectrum,
 * reduction partials, atom bins) is a caller allocation of
 * hartree_workspace_size() bytes handed over by hartree_bind_workspace().
 * Unless stated otherwise, pointers below are DEVICE pointers, arrays are
 * C-contiguous, and nothing is retained after a call returns.
 *
 * Execution: every compute call enqueues asynchronously on `stream` (a
 * hipStream_t; NULL means the default stream), performs no allocation and no
 * host synchronization, and returns once the work is enqueued.  A plan and its
 * workspace serve one stream at a time: two calls on one plan that overlap in
 * time race on the workspace.
 *
 * Errors: each call validates its arguments before enqueuing anything and
 * returns a status code; hartree_last_error() then describes the problem
 * (thread-local).  No C++ exception crosses this boundary.  A HIP launch
 * failure returns HARTREE_ERR_HIP.  Conditions that only the device can see
 * (a non-finite atom position, an atom wider than the plan's max_sigma, atom
 * bins overflowing) set bits in a device status word read by
 * hartree_device_status(); the affected outputs are then unspecified.
 */
#ifndef HARTREE_H
#define HARTREE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hartree_plan_s *hartree_plan;

typedef enum { HARTREE_FP64 = 0, HARTREE_FP32 = 1 } hartree_precision;

typedef enum {
    HARTREE_OK = 0,
    HARTREE_ERR_ARG = 1,         /* null pointer, negative count, bad enum, ... */
    HARTREE_ERR_DIMS = 2,        /* a grid dimension < 1, too large, or with a prime factor > 7 */
    HARTREE_ERR_CELL = 3,        /* non-finite cell or |det| too small */
    HARTREE_ERR_UNSUPPORTED = 4, /* valid input the library does not handle */
    HARTREE_ERR_WORKSPACE = 5,   /* no workspace bound, or the bound one is too small / misaligned */
    HARTREE_ERR_HIP = 6          /* a HIP runtime call failed */
} hartree_status;

/* Device status bits (hartree_device_status). */
#define HARTREE_DEV_BAD_ATOM 0x1u      /* non-finite position, sigma <= 0 or non-finite charge */
#define HARTREE_DEV_SIGMA_RANGE 0x2u   /* an atom's sigma exceeds the plan's max_sigma */
#define HARTREE_DEV_BIN_OVERFLOW 0x4u  /* atom bins exceeded their capacity */

/* Optional plan settings; zero fields take the defaults in brackets. */
typedef struct {
    double cutoff_sigmas; /* Gaussian truncation radius in units of sigma [FP32: 6; FP64: 8 when every
                             cell is diagonal (per-axis box), 9 otherwise (sphere)] */
    double max_sigma;     /* largest sigma the splat workspace is sized for, Bohr [1.0] */
    int32_t max_atoms;    /* largest atom count per splat call [65536] */
    int32_t reserved[7];  /* must be zero */
} hartree_plan_opts;

/* Create a plan for one periodic cell.
 *   cell  host, 9 doubles: the rows a, b, c (Bohr).  Any non-singular cell is
 *         accepted.  The splat calls use separable per-axis factors (and, in
 *         FP32, the matrix cores) in diagonal cells with positive edges, and a
 *         direct per-point evaluation in any other cell.
 *   dims  host, 3 int32: Na, Nb, Nc, each >= 1, <= 4096 and 7-smooth.
 *   precision  HARTREE_FP64 or HARTREE_FP32.
 *   opts  host, nullable.
 * On success *out receives the plan (host memory owned by the library until
 * hartree_plan_destroy). */
hartree_status hartree_plan_create(hartree_plan *out, const double cell[9], const int32_t dims[3],
                                   int32_t precision, const hartree_plan_opts *opts);

/* Create a plan for nprob independent cells solved together (the batched
 * workload: many densities on uneven grids).  cells: host, nprob x 9 doubles;
 * dims: host, nprob x 3 int32.  Grid arrays of a batched plan are the
 * problems' grids concatenated in problem order (offsets from
 * hartree_plan_grid_offset); energies are nprob doubles. */
hartree_status hartree_plan_create_batched(hartree_plan *out, int32_t nprob, const double *cells,
                                           const int32_t *dims, int32_t precision,
                                           const hartree_plan_opts *opts);

void hartree_plan_destroy(hartree_plan plan);

/* Number of problems (1 for a single plan) and the element offset of problem
 * p's grid in a concatenated grid array; offset(nprob) is the total. */
hartree_status hartree_plan_nprob(hartree_plan plan, int32_t *nprob);
hartree_status hartree_plan_grid_offset(hartree_plan plan, int32_t p, int64_t *offset);

/* Workspace: bytes needed (host out), then bind a device allocation of at
 * least that many bytes, 256-byte aligned.  Binding uploads the FP64-generated
 * twiddle tables with a synchronous copy; apart from hartree_device_status,
 * hartree_plan_set_config and hartree_plan_tune it is the only call that
 * synchronizes.  Rebinding replaces the previous workspace.  The first binding
 * also creates four internal streams of default priority on the current
 * device.  Work forked onto them (the launch groups of a batched plan's
 * transform passes, i.e. problems with different pass shapes that no single
 * multi-plan launch takes, and the backward chain of
 * hartree_solve_backward) starts
 * after the work already queued on the caller's stream and is joined back
 * before the call returns, so calls stay ordered on the caller's stream
 * (under capture the forked work becomes parallel branches of the graph).
 * If the streams cannot be created everything runs on the caller's stream;
 * results are the same either way.  The plan owns the streams until
 * hartree_plan_destroy. */
hartree_status hartree_workspace_size(hartree_plan plan, size_t *bytes);
hartree_status hartree_bind_workspace(hartree_plan plan, void *workspace, size_t bytes);

/* Hartree potential and energy, Eq. (6) and the E_Hartree term of Eq. (7)
 * (Sec. 2.1), on the periodic grid with the G = 0 term dropped:
 *   V = F^-1 [K F rho],  K(G) = 4 pi / |G|^2,  K(0) = 0,
 *   E_H = 1/2 sum_r rho(r) V(r) dV,  dV = |det cell| / (Na Nb Nc).
 * rho (in) and v (out) are grids of the plan's precision; v may not alias
 * rho.  e_h (nullable) receives E_H as double (one per problem).  The
 * transform runs along c, then b, then a and back, the layout order of
 * Sec. 3.2.4.  On an even axis the Nyquist index is taken as the average of
 * its two aliases (+N/2 and -N/2), which keeps the operator symmetric in any
 * cell. */
hartree_status hartree_solve(hartree_plan plan, const void *rho, void *v, double *e_h, void *stream);

/* E_H only (the forward half of the transform; no potential written). */
hartree_status hartree_energy(hartree_plan plan, const void *rho, double *e_h, void *stream);

/* Gradient of a loss L(V, E_H) with respect to rho, given the upstream
 * gradients grad_v = dL/dV (grid, nullable = zero) and grad_e = dL/dE_H
 * (device doubles, one per problem, nullable = zero):
 *   grad_rho = P (grad_v + grad_e * dV * rho),  P = F^-1 K F symmetric.
 * rho may be NULL only when grad_e is NULL.  grad_rho may not alias the
 * inputs.  Not in the paper: it follows from the symmetry of P. */
hartree_status hartree_backward(hartree_plan plan, const void *grad_v, const double *grad_e, const void *rho,
                                void *grad_rho, void *stream);

/* hartree_solve and hartree_backward in one call, for a loss whose upstream
 * gradients grad_v and grad_e are known before the solve (a loss linear in V
 * and E_H, or a step that reuses the previous gradients): the backward
 * chain needs only rho, grad_v and grad_e, not V, so the two chains of five
 * passes run side by side: the solve's on a stream of the plan's own,
 * forked from `stream` after the work already on it and joined back into it
 * before the call returns (under capture: a parallel branch of the graph),
 * the backward's on `stream` with its own spectrum buffer (the workspace's
 * last part).  Results are
 * identical to the two calls in order.  Arguments as in the two calls; v may
 * in addition not alias grad_v or grad_rho.  The chains run side by side
 * when their two spectra fit the 256 MiB last-level cache together and every
 * pass of the plan is one launch group (single plans, and batched plans
 * whose problems all take multi-plan launches); otherwise, or without the
 * plan's side streams, in order on `stream` (a spectrum that fits the cache
 * alone then stays there between passes). */
hartree_status hartree_solve_backward(hartree_plan plan, const void *rho, void *v, double *e_h, const void *grad_v,
                                      const double *grad_e, void *grad_rho, void *stream);

/* Gaussian atomic density on the grid (stands in for the density of Eq. (9)):
 *   rho(r) = sum_a Z_a (2 pi s_a^2)^(-3/2) sum_L exp(-|r - R_a - L|^2 / (2 s_a^2))  [- Q / Omega]
 * over lattice vectors L, truncated at cutoff_sigmas * s_a (per axis in a
 * diagonal cell, a sphere in any other cell); Q = sum Z_a.
 *   natoms  atom count (host int; for a batched plan the total over problems),
 *   pos     natoms x 3 Cartesian positions (any, wrapped into the cell),
 *   Z, sigma  natoms charges and widths (sigma > 0, <= max_sigma),
 *   atom_offsets  batched plans only: host, nprob + 1 int32 prefix offsets of
 *           each problem's atoms (NULL for single plans),
 *   rho_out grid of the plan's precision (overwritten),
 *   subtract_background  nonzero subtracts Q / Omega (a neutral cell).
 * Any cell (see hartree_plan_create). */
hartree_status hartree_splat(hartree_plan plan, int32_t natoms, const double *pos, const double *Z,
                             const double *sigma, const int32_t *atom_offsets, void *rho_out,
                             int32_t subtract_background, void *stream);

/* Adjoint of the splat with respect to atom positions:
 *   grad_pos[a] = sum_r grad_rho(r) d rho(r) / d R_a
 *               = Z_a (2 pi s_a^2)^(-3/2) / s_a^2 sum_r grad_rho(r) sum_L g(d) d,
 *   d = r - R_a - L,  g(d) = exp(-|d|^2 / (2 s_a^2)),
 * with the splat's truncation.  With grad_rho = dV * V this is dE_H/dR_a, the
 * negative Hartree force (the Hartree part of the forces of Sec. 5.2.5).
 * grad_pos: natoms x 3 doubles (overwritten).  Summation order is fixed, so
 * results are bitwise reproducible for a given plan. */
hartree_status hartree_splat_adjoint(hartree_plan plan, int32_t natoms, const double *pos, const double *Z,
                                     const double *sigma, const int32_t *atom_offsets, const void *grad_rho,
                                     double *grad_pos, void *stream);

/* Kernel groups timed by the profiling calls below. */
typedef enum {
    HARTREE_K_R2C = 0,        /* P1 forward: r2c along c */
    HARTREE_K_R2C_BWD = 1,    /* P1 backward: forms grad_v + grad_e dV rho, r2c along c */
    HARTREE_K_FFT_B = 2,      /* P2: FFT along b */
    HARTREE_K_FFT_A = 3,      /* P3 with the E_H partials: FFT along a, x K/N, inverse along a */
    HARTREE_K_FFT_A_BWD = 4,  /* P3 without the energy (backward, or no e_h requested) */
    HARTREE_K_FFT_A_EONLY = 5,/* P3 of hartree_energy: FFT along a and the E_H partials */
    HARTREE_K_FFT_B_INV = 6,  /* P4: inverse FFT along b */
    HARTREE_K_C2R = 7,        /* P5: c2r along c */
    HARTREE_K_FINALIZE = 8,   /* E_H fixed-order reduction */
    HARTREE_K_BIN = 9,        /* atom binning (prep, count, scan, fill, sort) */
    HARTREE_K_SPLAT = 10,     /* splat gather */
    HARTREE_K_ADJOINT = 11,   /* splat adjoint per-brick partials */
    HARTREE_K_ADJOINT_FINAL = 12, /* per-atom fixed-order reduction */
    HARTREE_K_COUNT = 13
} hartree_kernel_id;

/* Profiling: between begin and end every kernel group enqueued by this plan is
 * bracketed by HIP events on its stream.  end waits for the last event and
 * writes, per hartree_kernel_id, the summed duration in milliseconds and the
 * number of launches (host arrays of HARTREE_K_COUNT entries). */
hartree_status hartree_profile_begin(hartree_plan plan);
hartree_status hartree_profile_end(hartree_plan plan, double *total_ms, int64_t *launches);

/* Atom binning shared by a splat and its adjoint.  hartree_splat and
 * hartree_splat_adjoint each bin their atoms into bricks of the grid (sorted
 * per-brick lists with per-slot atom records in the workspace) before
 * their main kernels.  When both run on the same atoms -- a forward splat and
 * the backward pass of the same positions -- the binning can be done once:
 *   hartree_atoms_bind  bins the atoms (same arguments as hartree_splat) and
 *                       returns a token (host out) naming this binding;
 *   hartree_splat_bound / hartree_splat_adjoint_bound  run on the binding
 *                       named by the token, and return HARTREE_ERR_ARG when
 *                       the workspace has been rebound since (any bind, or an
 *                       unbound splat or adjoint call, replaces the binding).
 * The atom arrays must not change on the device while a binding is used. */
hartree_status hartree_atoms_bind(hartree_plan plan, int32_t natoms, const double *pos, const double *Z,
                                  const double *sigma, const int32_t *atom_offsets, uint64_t *token, void *stream);
hartree_status hartree_splat_bound(hartree_plan plan, uint64_t token, void *rho_out, int32_t subtract_background,
                                   void *stream);
hartree_status hartree_splat_adjoint_bound(hartree_plan plan, uint64_t token, const void *grad_rho, double *grad_pos,
                                           void *stream);

/* Size of the last binding (by hartree_atoms_bind, hartree_splat or
 * hartree_splat_adjoint): the number of (atom, brick) pairs in the per-brick
 * lists, i.e. the work of the splat and adjoint kernels.  Read synchronously
 * from the workspace after the work on `stream`; HARTREE_ERR_ARG during a
 * graph capture or for a NULL pointer. */
hartree_status hartree_atoms_pairs(hartree_plan plan, int64_t *pairs, void *stream);

/* Read (synchronously) and clear the device status word (HARTREE_DEV_* bits).
 * Refused (HARTREE_ERR_ARG) while a graph capture is open on the plan. */
hartree_status hartree_device_status(hartree_plan plan, uint32_t *bits, void *stream);

/* One-launch replay of a whole step (not from the paper: it replaces per-call
 * launches by one HIP graph launch, e.g. for the batched workload of many
 * small problems).
 *   hartree_graph_begin  starts capturing `stream` (a created stream, not the
 *                        default one) in thread-local mode;
 *   then the caller enqueues any sequence of this plan's compute calls on that
 *   stream (for instance hartree_splat_bound, hartree_solve,
 *   hartree_backward, hartree_splat_adjoint_bound): they are recorded, not run;
 *   hartree_graph_end    ends the capture and instantiates the graph, which the
 *                        plan keeps (replacing an earlier one);
 *   hartree_graph_launch replays it on any stream.
 * A replay reads and writes the same device addresses as the captured calls
 * (current contents of the inputs, including atom positions of the binding
 * that was current at capture; the binding itself is recomputed only if
 * hartree_atoms_bind was among the captured calls).  Run the sequence once
 * without capture first: that first run makes the one-time attribute calls
 * that capture does not allow.  No profiling events are recorded while
 * capturing; hartree_bind_workspace and hartree_device_status are refused.
 * A HIP error inside the capture makes hartree_graph_end return
 * HARTREE_ERR_HIP and keep the previous graph. */
hartree_status hartree_graph_begin(hartree_plan plan, void *stream);
hartree_status hartree_graph_end(hartree_plan plan, void *stream);
hartree_status hartree_graph_launch(hartree_plan plan, void *stream);

/* Pass shapes: for every problem q and axis x (0 = a, 1 = b, 2 = c) a plan
 * uses a radix sequence (an entry of the library's compiled plan table, or -1
 * for the default factorization on the run-time radix kernel), a tile of
 * 2^p_log2 pencils per workgroup and, on the strided axes a and b, an LDS
 * pitch of 2^p_log2 + pad complex values (pad 0 .. 3; 0 on axis c).  cfg is a
 * host array of nprob x 3 x 3 int32: cfg[3 (3 q + x) + 0, 1, 2] = plan
 * entry, p_log2, pad.  The choice changes only the schedule and the rounding
 * order of the FP32/FP64 sums, not what is computed.
 *   hartree_plan_get_config  writes the current choice;
 *   hartree_plan_set_config  validates and applies one (HARTREE_ERR_ARG if an
 *                            entry does not factor the length, needs more
 *                            threads than a workgroup has, or more LDS than
 *                            the device allows); with a workspace bound it
 *                            re-uploads the problem descriptors (synchronous);
 *   hartree_plan_tune        times every valid choice per (axis, length), the
 *                            forward and inverse passes of that axis, `reps`
 *                            times each on `stream`, keeps the fastest and
 *                            applies it.  scratch: a device grid of the plan's
 *                            precision and total grid size, overwritten.
 *                            Synchronous; needs a bound workspace. */
hartree_status hartree_plan_get_config(hartree_plan plan, int32_t *cfg);
hartree_status hartree_plan_set_config(hartree_plan plan, const int32_t *cfg);
hartree_status hartree_plan_tune(hartree_plan plan, void *scratch, int32_t reps, void *stream);

/* Atom decomposition (Sec. 3.1): the modified recursive bisection (Sec. 3.1.2)
 * along inertia-tensor principal axes (Eq. (11)-(18)) with per-atom weights
 * (Eq. (19)), as laid out in Sec. 3.1.5.  Host code on HOST memory; no device
 * work, callable without a GPU.
 *   pos        natoms x 3 doubles, Cartesian positions (Bohr) as given: the
 *              cell is not consulted, so wrap periodic images first if the
 *              parts should be compact in the wrapped cell;
 *   weights    natoms doubles, each finite and > 0 (e.g. Etime_i / Mtime of
 *              Eq. (19)), or NULL for unit weights;
 *   nparts     number of parts (processes), >= 1, any value;
 *   order      out, natoms int32: atom indices grouped by part, parts in the
 *              order of the bisection tree's leaves (lower projection first),
 *              atoms inside a part in the order of their last projection;
 *   part       out, natoms int32: part of each atom, or NULL;
 *   part_start out, nparts + 1 int32: part p is order[part_start[p] ..
 *              part_start[p + 1]), or NULL.
 * A tree node with one part or no atoms is a leaf; otherwise its first
 * ceil(n/2) parts take the atoms of lowest projection on the axis that
 * maximises sum_i w_i t_i^2, as many as bring their weight nearest to that
 * share of the node's weight (ties: the lower side takes one more).  The
 * centre of Eq. (12) is normalised by the node's total weight, and the axis's
 * sign makes its largest component positive.  Parts may be empty when nparts
 * exceeds natoms.  Deterministic: ties in projection go by atom index.
 * HARTREE_ERR_ARG for a negative count, nparts < 1, a NULL pos (natoms > 0)
 * or order, a non-finite position, or a weight that is not finite and > 0. */
hartree_status hartree_atom_partition(int32_t natoms, const double *pos, const double *weights, int32_t nparts,
                                      int32_t *order, int32_t *part, int32_t *part_start);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as hartree_solve (V, and E_H when e_h is not NULL) with no
 * workspace bound to the plan and no allocation of any kind.  The plan's
 * problem descriptors, twiddle tables, half spectrum and E_H partials live in
 * a device array owned by the library, HARTREE_NOALLOC_BYTES (64 MiB) per
 * GPU, which every GPU the library runs on holds until the process ends; the
 * first call on a device looks up that device's copy (the current device's,
 * which must be the stream's).  Each call first rewrites the descriptors and
 * twiddles (twiddles generated on the device in FP64, so an FP64 plan may
 * differ from hartree_solve in the last bit of a twiddle) and every
 * intermediate it reads, so nothing needs clearing between calls.
 *   rho, v, e_h, stream  as for hartree_solve; everything runs in order on
 *                        `stream` (no internal side streams).
 * HARTREE_ERR_WORKSPACE, before anything is enqueued, when the plan needs more
 * than HARTREE_NOALLOC_BYTES (the message names both sizes): a 240^3 FP32 or
 * a 180^3 FP64 plan fits, a 256^3 FP32 plan does not.  All calls on one GPU
 * share the one array: two calls that overlap in time on the same GPU (two
 * streams, two threads, or a call beside a graph replay that contains one)
 * race on it and give wrong results; a caller serializes them. */
#define HARTREE_NOALLOC_BYTES (64u * 1024u * 1024u)
hartree_status hartree_solve_noalloc(hartree_plan plan, const void *rho, void *v, double *e_h, void *stream);

/* Description of the last error on the calling thread ("" if none). */
const char *hartree_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HARTREE_H */
