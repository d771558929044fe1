// C ABI of the Hartree library: plan creation and validation, workspace
// layout, twiddle generation, and the enqueue of every pass.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hartree.h"
#include "fft_core.hpp"
#include "partition.hpp"
#include "kernels.hpp"

using namespace hartree;

namespace {

thread_local std::string g_last_error;

hartree_status fail(hartree_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
hartree_status fail(hartree_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

hartree_status ok()
{
    g_last_error.clear();
    return HARTREE_OK;
}

hartree_status hip_fail(hipError_t e, const char *what)
{
    return fail(HARTREE_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Stage radices for a length: the fewest stages over the butterfly radices
// the kernels implement, {16, 10, 9, 8, 7, 5, 4, 3, 2}; among those, the
// smallest largest radix, then the order found first (larger radices first).
constexpr int kRadices[] = {16, 10, 9, 8, 7, 5, 4, 3, 2};

// a plan fits when every stage's butterflies fit one workgroup's registers
bool plan_fits(int n, int fp64, const std::vector<int> &r)
{
    return pass_p_log2(fp64, n, r.data(), int(r.size()), 64) >= 0;
}

void factor_search(int n, int m, int fp64, std::vector<int> &cur, std::vector<int> &best)
{
    if (m == 1) {
        auto maxr = [](const std::vector<int> &v) {
            int x = 0;
            for (int y : v) x = y > x ? y : x;
            return x;
        };
        if (!plan_fits(n, fp64, cur)) return;
        if (best.empty() || cur.size() < best.size() || (cur.size() == best.size() && maxr(cur) < maxr(best)))
            best = cur;
        return;
    }
    if (!best.empty() && cur.size() + 1 > best.size()) return;
    if (int(cur.size()) >= kMaxStages) return;
    for (int r : kRadices) {
        if (m % r == 0) {
            cur.push_back(r);
            factor_search(n, m / r, fp64, cur, best);
            cur.pop_back();
        }
    }
}

bool factorize(int n, int fp64, std::vector<int> &r)
{
    r.clear();
    if (n == 1) return true;
    std::vector<int> cur;
    factor_search(n, n, fp64, cur, r);
    return !r.empty();
}

// cos and sin of 2 pi t / n with the angle reduced exactly to the first
// octant in integer arithmetic before calling std::cos / std::sin.
void unit_root(long t, long n, double &c, double &s)
{
    t %= n;
    if (t < 0) t += n;
    const long u = 4 * t;
    const long q = u / n;      // quadrant
    long r = u - q * n;        // angle within the quadrant: (pi/2) r / n
    bool swap = false;
    if (2 * r > n) {           // use the complement for the upper half of the quadrant
        r = n - r;
        swap = true;
    }
    const double th = 1.5707963267948966192313216916397514 * double(r) / double(n);
    double cc = std::cos(th), ss = std::sin(th);
    if (swap) std::swap(cc, ss);
    switch (q) {
    case 0: c = cc; s = ss; break;
    case 1: c = -ss; s = cc; break;
    case 2: c = -cc; s = -ss; break;
    default: c = ss; s = -cc; break;
    }
}

struct Launch {
    int plan;    // compiled radix plan (index in HARTREE_PLANS) or -1
    int p_log2;  // pencils per workgroup, log2
    int pad;     // LDS pitch pad of strided tiles
    int maxn;    // longest pencil in the launch (sizes the LDS tile)
    int64_t col_stride;  // largest pencil stride (elements) of the strided passes
    TileList tl;
};

}  // namespace

struct hartree_plan_s {
    int fp64 = 0;
    int nprob = 0;
    bool splat_ok = false;
    bool general = false;  // some cell needs the general-cell splat kernels
    double cutoff = 0.0;
    double max_sigma = 0.0;
    int max_atoms = 0;
    std::vector<ProbDesc> desc;
    std::vector<double> twiddles;  // interleaved (re, im), FP64
    int64_t spec_count = 0;        // complex elements
    int64_t grid_total = 0;        // real elements
    std::vector<int64_t> grid_offsets;
    int nparts = 0;
    int64_t nbricks = 0;
    int64_t capacity = 0;
    std::vector<Launch> lr2c, lb, la;  // P1/P5 (axis c), P2/P4 (axis b), P3 (axis a)
    // per problem and axis (a, b, c): compiled radix plan (-1: run-time
    // radix kernel), log2 of the pencils per workgroup, LDS pitch pad
    struct AxisCfg {
        int plan;
        int p_log2;
        int pad;
    };
    std::vector<AxisCfg> cfg;
    int64_t max_parts = 0;  // E_H partial slots at one pencil per workgroup
    // workspace layout
    size_t o_status = 0, o_desc = 0, o_tw = 0, o_spec = 0, o_parts = 0, o_qsum = 0, o_info = 0, o_counts = 0,
           o_offsets = 0, o_cursor = 0, o_list = 0, o_lists = 0, o_bpart = 0, o_slot = 0, o_rec = 0, o_order = 0, o_zero = 0,
           o_spec2 = 0, ws_size = 0;
    int32_t cap_pa = 0;
    bool wide = false;  // some truncation window can hold two images of one grid point
    unsigned char *ws = nullptr;
    // profiling: events bracketing each kernel group
    struct ProfRec {
        int id;
        hipEvent_t a, b;
    };
    bool prof = false;
    std::vector<hipEvent_t> pool;
    size_t pool_used = 0;
    std::vector<ProfRec> recs;
    // current atom binding (hartree_atoms_bind)
    uint64_t bind_token = 0;
    bool bound = false;
    int32_t bound_natoms = 0;
    const double *bound_pos = nullptr, *bound_Z = nullptr, *bound_sigma = nullptr;
    std::vector<int32_t> bound_offsets;
    // stream capture into a graph (hartree_graph_begin / end / launch)
    bool capturing = false;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    void drop_graph()
    {
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        if (graph) (void)hipGraphDestroy(graph);
        graph_exec = nullptr;
        graph = nullptr;
    }
    // side streams of a batched plan: the launch groups of one pass (problems
    // with different pass shapes) write disjoint problems, so they run side by
    // side, forked from and joined back into the caller's stream by events
    // (under capture: parallel branches of the graph).  Default priority.
    static constexpr int kSide = 3;
    hipStream_t side[kSide] = {};
    hipEvent_t fork_ev = nullptr;
    hipEvent_t join_ev[kSide] = {};
    // hartree_solve_backward runs one of its two chains on this stream (a
    // parallel branch beside the other, each on its own spectrum buffer),
    // forked from and joined back into the caller's stream
    hipStream_t chain_side = nullptr;
    hipEvent_t chain_fork = nullptr, chain_join = nullptr;
    bool side_ready = false;
    void drop_side()
    {
        for (int i = 0; i < kSide; ++i) {
            if (side[i]) (void)hipStreamDestroy(side[i]);
            if (join_ev[i]) (void)hipEventDestroy(join_ev[i]);
            side[i] = nullptr;
            join_ev[i] = nullptr;
        }
        if (chain_side) (void)hipStreamDestroy(chain_side);
        chain_side = nullptr;
        for (hipEvent_t *q : {&fork_ev, &chain_fork, &chain_join}) {
            if (*q) (void)hipEventDestroy(*q);
            *q = nullptr;
        }
        side_ready = false;
    }
    ~hartree_plan_s()
    {
        drop_graph();
        drop_side();
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

namespace {

bool is_smooth(int n)
{
    if (n < 1 || n > kMaxN) return false;
    for (int p : {2, 3, 5, 7})
        while (n % p == 0) n /= p;
    return n == 1;
}

void add_launch(std::vector<Launch> &v, int plan, int p_log2, int pad, int n, int64_t col_stride, int prob, int tiles)
{
    for (auto &l : v) {
        if (l.plan == plan && l.p_log2 == p_log2 && l.pad == pad && l.tl.count < kMaxProb) {
            l.tl.prob[l.tl.count] = prob;
            l.tl.start[l.tl.count + 1] = l.tl.start[l.tl.count] + tiles;
            l.tl.count++;
            l.tl.total += tiles;
            if (n > l.maxn) l.maxn = n;
            if (col_stride > l.col_stride) l.col_stride = col_stride;
            return;
        }
    }
    Launch l;
    std::memset(&l, 0, sizeof(l));
    l.plan = plan;
    l.p_log2 = p_log2;
    l.pad = pad;
    l.maxn = n;
    l.col_stride = col_stride;
    l.tl.count = 1;
    l.tl.prob[0] = prob;
    l.tl.start[0] = 0;
    l.tl.start[1] = tiles;
    l.tl.total = tiles;
    v.push_back(l);
}

// launch groups of the three pass kinds and the E_H partial slots from the
// per-axis choices in p->cfg
// The multi-plan launch shape of axis x (FP32 batched plans), or -1: every
// problem on a plan of the axis' multi-plan list with no pitch pad and either
// one common tile width of the fixed shapes (returns its log2) or each at its
// length's size-adapted width (returns kMultiAutoLog); on the strided axes
// the lanes' byte offsets must fit 32 bits.
int multi_axis(hartree_plan p, int x)
{
    if (p->nprob < 2 || p->fp64) return -1;
    const int lp0 = p->cfg[x].p_log2;
    bool common = lp0 == multi_log_p(x, 0) || lp0 == multi_log_p(x, 1), sized = true;
    const int *list = multi_plans(x);
    for (int q = 0; q < p->nprob; ++q) {
        const auto &c = p->cfg[3 * q + x];
        if (std::find(list, list + kMultiPlans, c.plan) == list + kMultiPlans || c.pad != 0) return -1;
        const ProbDesc &d = p->desc[q];
        common = common && c.p_log2 == lp0;
        sized = sized && (1 << c.p_log2) == multi_auto_p(d.dims[x], x);
        if (x < 2) {
            // the compiled strided tiles address lanes with 32-bit byte offsets
            const int64_t st = x == 0 ? int64_t(d.dims[1]) * d.dims[3] : d.dims[3];
            const int64_t P = int64_t(1) << c.p_log2, tpp = 256 / P;  // 256 threads per pass workgroup
            if (((tpp - 1) * st + P) * 8 >= (int64_t(1) << 32)) return -1;
        }
    }
    if (common) return lp0;
    return sized ? kMultiAutoLog : -1;
}

void rebuild_launches(hartree_plan p)
{
    p->lr2c.clear();
    p->lb.clear();
    p->la.clear();
    p->nparts = 0;
    int multi[3];
    for (int x = 0; x < 3; ++x) multi[x] = multi_axis(p, x);
    for (int q = 0; q < p->nprob; ++q) {
        ProbDesc &d = p->desc[q];
        const auto *c = &p->cfg[3 * q];
        for (int x = 0; x < 3; ++x) d.ax[x].cplan = c[x].plan;
        const int pa = 1 << c[0].p_log2, pb = 1 << c[1].p_log2, pc = 1 << c[2].p_log2;
        const int64_t rows = int64_t(d.dims[0]) * d.dims[1];
        const int64_t t1 = (rows + 2 * pc - 1) / (2 * pc);
        const int64_t t2 = int64_t(d.dims[0]) * ((d.dims[3] + pb - 1) / pb);
        const int64_t t3 = (int64_t(d.dims[1]) * d.dims[3] + pa - 1) / pa;
        // a multi-plan axis puts every problem in one launch group (the
        // kernel reads each problem's plan from its descriptor)
        // (launch shape: the common tile width, or kMultiAutoLog for tiles
        // sized per length; the tile counts above use each problem's own)
        auto shape = [&](int x) { return multi[x] >= 0 ? multi[x] : c[x].p_log2; };
        add_launch(p->lr2c, multi[2] >= 0 ? kMultiPlan : c[2].plan, shape(2), c[2].pad, d.dims[2], 0, q, int(t1));
        add_launch(p->lb, multi[1] >= 0 ? kMultiPlan : c[1].plan, shape(1), c[1].pad, d.dims[1], d.dims[3], q, int(t2));
        add_launch(p->la, multi[0] >= 0 ? kMultiPlan : c[0].plan, shape(0), c[0].pad, d.dims[0],
                   int64_t(d.dims[1]) * d.dims[3], q, int(t3));
        d.part_off = p->nparts;
        d.nparts = int(t3);
        p->nparts += int(t3);
    }
}

hartree_status create(hartree_plan *out, int nprob, const double *cells, const int32_t *dims, int32_t precision,
                      const hartree_plan_opts *opts)
{
    if (!out) return fail(HARTREE_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!cells || !dims) return fail(HARTREE_ERR_ARG, "cell or dims is NULL");
    if (nprob < 1 || nprob > kMaxProb) return fail(HARTREE_ERR_ARG, "nprob must be in [1, %d]", kMaxProb);
    if (precision != HARTREE_FP64 && precision != HARTREE_FP32)
        return fail(HARTREE_ERR_ARG, "precision must be HARTREE_FP64 or HARTREE_FP32");
    hartree_plan_opts opt;
    std::memset(&opt, 0, sizeof(opt));
    if (opts) {
        opt = *opts;
        for (int i = 0; i < 7; ++i)
            if (opt.reserved[i] != 0) return fail(HARTREE_ERR_ARG, "opts.reserved must be zero");
        if (!(opt.cutoff_sigmas >= 0.0) || !(opt.max_sigma >= 0.0) || opt.max_atoms < 0)
            return fail(HARTREE_ERR_ARG, "negative or NaN option");
    }
    auto p = new hartree_plan_s();
    p->fp64 = precision == HARTREE_FP64;
    p->nprob = nprob;
    // Default truncation: 6 sigma in FP32; in FP64 8 sigma where the cutoff
    // is a per-axis box (diagonal cells) and 9 sigma where it is a sphere
    // (any other cell in the plan): the sphere leaves out the box's corners,
    // and at 8 sigma its omitted tails reach 1e-13 of the density's maximum
    // in dense lattices (2.8e-16 at 9 sigma).
    bool any_general = false;
    for (int q = 0; q < nprob; ++q) {
        const double *A = cells + 9 * q;
        const bool diag = A[1] == 0.0 && A[2] == 0.0 && A[3] == 0.0 && A[5] == 0.0 && A[6] == 0.0 && A[7] == 0.0;
        if (!(diag && A[0] > 0.0 && A[4] > 0.0 && A[8] > 0.0)) any_general = true;
    }
    p->cutoff = opt.cutoff_sigmas > 0.0 ? opt.cutoff_sigmas : (p->fp64 ? (any_general ? 9.0 : 8.0) : 6.0);
    p->max_sigma = opt.max_sigma > 0.0 ? opt.max_sigma : 1.0;
    p->max_atoms = opt.max_atoms > 0 ? opt.max_atoms : 65536;
    p->desc.resize(nprob);
    std::map<int, int> tw_off;
    p->splat_ok = true;
    int64_t grid = 0, spec = 0, bricks = 0;
    int64_t cap_per_atom = 0;
    for (int q = 0; q < nprob; ++q) {
        const double *A = cells + 9 * q;
        const int32_t *N = dims + 3 * q;
        for (int x = 0; x < 3; ++x) {
            if (!is_smooth(N[x])) {
                delete p;
                return fail(HARTREE_ERR_DIMS, "problem %d: dimension %d is %d; need 1..%d with prime factors 2, 3, 5, 7",
                            q, x, N[x], kMaxN);
            }
        }
        for (int i = 0; i < 9; ++i) {
            if (!std::isfinite(A[i])) {
                delete p;
                return fail(HARTREE_ERR_CELL, "problem %d: non-finite cell entry", q);
            }
        }
        const double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                           A[2] * (A[3] * A[7] - A[4] * A[6]);
        const double n0 = std::sqrt(A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
        const double n1 = std::sqrt(A[3] * A[3] + A[4] * A[4] + A[5] * A[5]);
        const double n2 = std::sqrt(A[6] * A[6] + A[7] * A[7] + A[8] * A[8]);
        if (!(std::fabs(det) > 1e-10 * n0 * n1 * n2) || !(std::fabs(det) > 0.0)) {
            delete p;
            return fail(HARTREE_ERR_CELL, "problem %d: singular or degenerate cell (det %g)", q, det);
        }
        ProbDesc &d = p->desc[q];
        std::memset(&d, 0, sizeof(d));
        for (int x = 0; x < 3; ++x) {
            const int n = N[x];
            AxisPlan &ap = d.ax[x];
            std::vector<int> rad;
            if (!factorize(n, p->fp64, rad)) {
                delete p;
                return fail(HARTREE_ERR_DIMS, "problem %d: cannot factor %d", q, n);
            }
            ap.n = n;
            ap.nstages = int(rad.size());
            int ns = 1;
            for (size_t s = 0; s < rad.size(); ++s) {
                ap.radix[s] = rad[s];
                ap.ns[s] = make_fastdiv(uint32_t(ns));
                ap.twstride[s] = n / (ns * rad[s]);
                ns *= rad[s];
            }
            auto it = tw_off.find(n);
            if (it == tw_off.end()) {
                const int off = int(p->twiddles.size() / 2);
                tw_off[n] = off;
                for (int t = 0; t < n; ++t) {
                    double c, s;
                    unit_root(t, n, c, s);
                    p->twiddles.push_back(c);
                    p->twiddles.push_back(-s);  // W_n^t = exp(-2 pi i t / n)
                }
                ap.tw_off = off;
            } else {
                ap.tw_off = it->second;
            }
        }
        d.dims[0] = N[0];
        d.dims[1] = N[1];
        d.dims[2] = N[2];
        d.dims[3] = N[2] / 2 + 1;
        d.div_nh = make_fastdiv(uint32_t(d.dims[3]));
        d.div_nc = make_fastdiv(uint32_t(N[2]));
        d.npts = int64_t(N[0]) * N[1] * N[2];
        d.grid_off = grid;
        d.spec_off = spec;
        p->grid_offsets.push_back(grid);
        grid += d.npts;
        spec += int64_t(N[0]) * N[1] * d.dims[3];
        // B = 2 pi inv(A)^T: row i = 2 pi (a_j x a_k) / det
        const double *a0 = A, *a1 = A + 3, *a2 = A + 6;
        const double c12[3] = {a1[1] * a2[2] - a1[2] * a2[1], a1[2] * a2[0] - a1[0] * a2[2],
                               a1[0] * a2[1] - a1[1] * a2[0]};
        const double c20[3] = {a2[1] * a0[2] - a2[2] * a0[1], a2[2] * a0[0] - a2[0] * a0[2],
                               a2[0] * a0[1] - a2[1] * a0[0]};
        const double c01[3] = {a0[1] * a1[2] - a0[2] * a1[1], a0[2] * a1[0] - a0[0] * a1[2],
                               a0[0] * a1[1] - a0[1] * a1[0]};
        const double tp = 6.283185307179586476925286766559;
        for (int k = 0; k < 3; ++k) {
            d.B[k] = tp * c12[k] / det;
            d.B[3 + k] = tp * c20[k] / det;
            d.B[6 + k] = tp * c01[k] / det;
        }
        for (int k = 0; k < 9; ++k) d.Bf[k] = float(d.B[k]);
        const bool ortho = A[1] == 0.0 && A[2] == 0.0 && A[3] == 0.0 && A[5] == 0.0 && A[6] == 0.0 && A[7] == 0.0;
        d.ortho = ortho ? 1 : 0;
        const double omega = std::fabs(det);
        d.inv_n = 1.0 / double(d.npts);
        d.dv = omega / double(d.npts);
        d.eh_scale = omega / (2.0 * double(d.npts) * double(d.npts));
        d.L[0] = A[0];
        d.L[1] = A[4];
        d.L[2] = A[8];
        for (int k = 0; k < 3; ++k) {
            d.h[k] = d.L[k] / double(d.dims[k]);
            d.hf[k] = float(d.h[k]);
            d.hfl[k] = float(d.h[k] - double(d.hf[k]));
        }
        for (int k = 0; k < 9; ++k) d.A[k] = A[k];
        d.separable = (ortho && A[0] > 0.0 && A[4] > 0.0 && A[8] > 0.0) ? 1 : 0;
        if (!d.separable) p->general = true;
        // pass tiles: default radix plan and pencils per workgroup per axis
        for (int x = 0; x < 3; ++x) {
            // strided axes (a, b): up to 64 pencils side by side; the c axis:
            // at most 4 pencils, so that a wavefront streams whole rows
            const int lp = pass_p_log2(p->fp64, N[x], d.ax[x].radix, d.ax[x].nstages, x == 2 ? 4 : 64);
            if (lp < 0) {
                delete p;
                return fail(HARTREE_ERR_DIMS, "problem %d: length %d needs more threads per pencil than a workgroup has",
                            q, N[x]);
            }
            // strided axes: the LDS pitch pad with the fewest modelled bank
            // conflicts, among those no larger in LDS than a pad of one
            int pad = 0;
            if (x < 2) {
                pad = pass_default_pad(p->fp64, N[x], d.ax[x].radix, d.ax[x].nstages, lp);
                if (pass_tile_lds(p->fp64, N[x], lp, pad) > pass_tile_lds(p->fp64, N[x], lp, 1)) pad = 1;
            }
            p->cfg.push_back({find_plan(d.ax[x].radix, d.ax[x].nstages), lp, pad});
        }
        // tile counts at one pencil per workgroup bound every choice
        const int64_t rows = int64_t(N[0]) * N[1];
        // (pass kernels also index one problem's half spectrum with 32-bit offsets)
        if ((rows + 1) / 2 > (1 << 30) || int64_t(N[0]) * d.dims[3] > (1 << 30) ||
            int64_t(N[1]) * d.dims[3] > (1 << 30) || rows * d.dims[3] >= (int64_t(1) << 31)) {
            delete p;
            return fail(HARTREE_ERR_DIMS, "problem %d: grid too large", q);
        }
        p->max_parts += int64_t(N[1]) * d.dims[3];
        // splat bricks
        // (FP64 plans with a non-diagonal cell keep the smaller bricks of the
        // point-by-point kernels)
        const bool small = p->fp64 && any_general;
        const int bsz[3] = {small ? kBI : kMI, small ? kBJ : kMJ, small ? kBK : kMK};
        int64_t per_atom = 1;
        for (int x = 0; x < 3; ++x) {
            d.bsz[x] = bsz[x];
            d.nbricks[x] = (N[x] + bsz[x] - 1) / bsz[x];
            // spacing of the grid planes across axis x: 2 pi / (|b_x| N_x)
            // (the edge length / N_x in a diagonal cell)
            const double bn = std::sqrt(d.B[3 * x] * d.B[3 * x] + d.B[3 * x + 1] * d.B[3 * x + 1] +
                                        d.B[3 * x + 2] * d.B[3 * x + 2]);
            const double h = 6.283185307179586476925286766559 / (bn * N[x]);
            const double w = std::floor(2.0 * p->cutoff * p->max_sigma / h) + 1.0;
            if (w + 1.0 > N[x]) p->wide = true;  // window points (+1 for rounding) exceed the axis
            int64_t nbx = d.nbricks[x];  // most bricks one atom's window touches along x
            if (w < N[x]) {
                const int64_t bnd = int64_t(std::ceil((w - 1.0) / bsz[x])) + 2;
                if (bnd < nbx) nbx = bnd;
            }
            per_atom *= nbx;
        }
        d.brick_off = bricks;
        bricks += int64_t(d.nbricks[0]) * d.nbricks[1] * d.nbricks[2];
        if (per_atom > cap_per_atom) cap_per_atom = per_atom;
    }
    p->grid_offsets.push_back(grid);
    p->grid_total = grid;
    p->spec_count = spec;
    rebuild_launches(p);
    p->nbricks = p->splat_ok ? bricks : 0;
    p->capacity = p->splat_ok ? int64_t(p->max_atoms) * cap_per_atom : 0;
    p->cap_pa = int32_t(cap_per_atom);
    if (p->capacity > int64_t(INT32_MAX)) {
        const int64_t cap = p->capacity;
        delete p;
        return fail(HARTREE_ERR_ARG, "splat bins (%lld entries) exceed 2^31; lower max_atoms or max_sigma",
                    (long long)cap);
    }
    // workspace layout
    const size_t cx = p->fp64 ? 16 : 8;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    p->o_status = take(sizeof(DeviceStatus));
    p->o_zero = take(256);
    p->o_desc = take(sizeof(ProbDesc) * nprob);
    p->o_tw = take(cx * (p->twiddles.size() / 2));
    p->o_spec = take(cx * size_t(p->spec_count));
    p->o_parts = take(8 * size_t(p->max_parts + 1));
    p->o_qsum = take(16 * size_t(nprob));  // per problem: the charge Q, then the largest atom weight
    if (p->splat_ok) {
        p->o_info = take(sizeof(AtomInfo) * size_t(p->max_atoms));
        p->o_counts = take(4 * size_t(p->nbricks + 1));
        p->o_offsets = take(4 * size_t(p->nbricks + 1));
        p->o_cursor = take(4 * size_t(p->nbricks + 1));
        p->o_list = take(4 * size_t(p->capacity));
        p->o_lists = take(4 * size_t(p->capacity));
        p->o_bpart = take(24 * size_t(p->capacity));
        p->o_slot = take(4 * size_t(p->capacity));
        if (!p->general) p->o_rec = take((p->fp64 ? sizeof(SlotAtom64) : sizeof(SlotAtom)) * size_t(p->capacity));
        if (nprob > 1) p->o_order = take(4 * size_t(p->nbricks));
    }
    // the second spectrum (hartree_solve_backward's backward chain), last,
    // so that the solve's part of the layout is the same with or without it
    p->o_spec2 = take(cx * size_t(p->spec_count));
    p->ws_size = o;
    *out = p;
    return ok();
}

hartree_status check_ws(hartree_plan p)
{
    if (!p) return fail(HARTREE_ERR_ARG, "plan is NULL");
    if (!p->ws) return fail(HARTREE_ERR_WORKSPACE, "no workspace bound (hartree_bind_workspace)");
    return HARTREE_OK;
}

constexpr size_t kMaxProfRecs = 1 << 16;

hipEvent_t next_event(hartree_plan p)
{
    if (p->pool_used == p->pool.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        p->pool.push_back(e);
    }
    return p->pool[p->pool_used++];
}

// run f(); while profiling, bracket it with events on stream s
template <typename F>
hipError_t timed(hartree_plan p, int id, hipStream_t s, F f)
{
    if (!p->prof || p->capturing || p->recs.size() >= kMaxProfRecs) return f();
    hipEvent_t a = next_event(p), b = next_event(p);
    if (!a || !b) return f();
    hipError_t e = hipEventRecord(a, s);
    if (e != hipSuccess) return e;
    e = f();
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, s);
    if (e != hipSuccess) return e;
    p->recs.push_back({id, a, b});
    return hipSuccess;
}

// pass arguments on a workspace laid out as the plan's (the bound one, or
// the no-allocation entry point's device scratch)
PassArgs base_args_at(hartree_plan p, unsigned char *ws)
{
    PassArgs a;
    std::memset(&a, 0, sizeof(a));
    a.desc = reinterpret_cast<const ProbDesc *>(ws + p->o_desc);
    a.tw = ws + p->o_tw;
    a.spec = ws + p->o_spec;
    a.partials = reinterpret_cast<double *>(ws + p->o_parts);
    return a;
}

PassArgs base_args(hartree_plan p) { return base_args_at(p, p->ws); }

int kernel_id(PassKind kind)
{
    switch (kind) {
    case PASS_R2C_FWD: return HARTREE_K_R2C;
    case PASS_R2C_BWD: return HARTREE_K_R2C_BWD;
    case PASS_C2R: return HARTREE_K_C2R;
    case PASS_B_FWD: return HARTREE_K_FFT_B;
    case PASS_B_INV: return HARTREE_K_FFT_B_INV;
    case PASS_A_FULL: return HARTREE_K_FFT_A;
    case PASS_A_NOENERGY: return HARTREE_K_FFT_A_BWD;
    default: return HARTREE_K_FFT_A_EONLY;
    }
}

// The launch groups of one pass.  With side streams (batched plans) the
// groups are dealt, largest first, to the least-loaded of the caller's stream
// and the side streams, forked after the work already on `s` and joined back
// before the pass returns; results do not depend on the dealing (disjoint
// problems, fixed per-problem sums).
hipError_t run_group(hartree_plan p, const std::vector<Launch> &groups, PassKind kind, PassArgs a, hipStream_t s)
{
    return timed(p, kernel_id(kind), s, [&]() -> hipError_t {
        const int ng = int(groups.size());
        const int nside = (ng > 1 && p->side_ready) ? std::min(ng - 1, int(hartree_plan_s::kSide)) : 0;
        if (nside == 0) {
            for (const Launch &l : groups) {
                a.tl = l.tl;
                a.col_stride = l.col_stride;
                hipError_t e = run_pass(p->fp64, kind, l.plan, l.p_log2, l.pad, l.maxn, l.tl.total, s, a);
                if (e != hipSuccess) return e;
            }
            return hipSuccess;
        }
        std::vector<int> order(ng);
        for (int i = 0; i < ng; ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(),
                         [&](int x, int y) { return groups[x].tl.total > groups[y].tl.total; });
        hipStream_t st[hartree_plan_s::kSide + 1] = {s};
        int64_t load[hartree_plan_s::kSide + 1] = {};
        for (int k = 0; k < nside; ++k) st[k + 1] = p->side[k];
        hipError_t e = hipEventRecord(p->fork_ev, s);
        for (int k = 0; k < nside && e == hipSuccess; ++k) e = hipStreamWaitEvent(p->side[k], p->fork_ev, 0);
        for (int i = 0; i < ng && e == hipSuccess; ++i) {
            int best = 0;
            for (int k = 1; k <= nside; ++k)
                if (load[k] < load[best]) best = k;
            const Launch &l = groups[order[i]];
            load[best] += l.tl.total;
            a.tl = l.tl;
            a.col_stride = l.col_stride;
            e = run_pass(p->fp64, kind, l.plan, l.p_log2, l.pad, l.maxn, l.tl.total, st[best], a);
        }
        // join every side stream that was forked, also after an error, so
        // that no capture is left with an unjoined branch
        for (int k = 0; k < nside; ++k) {
            hipError_t j = hipEventRecord(p->join_ev[k], p->side[k]);
            if (j == hipSuccess) j = hipStreamWaitEvent(s, p->join_ev[k], 0);
            if (e == hipSuccess) e = j;
        }
        return e;
    });
}

SplatArgs splat_args(hartree_plan p, int32_t natoms, const double *pos, const double *Z, const double *sigma,
                     const int32_t *atom_offsets)
{
    SplatArgs a;
    std::memset(&a, 0, sizeof(a));
    a.desc = reinterpret_cast<const ProbDesc *>(p->ws + p->o_desc);
    a.nprob = p->nprob;
    a.natoms = natoms;
    if (p->nprob == 1) {
        a.atom_off[0] = 0;
        a.atom_off[1] = natoms;
    } else {
        for (int i = 0; i <= p->nprob; ++i) a.atom_off[i] = atom_offsets[i];
    }
    a.pos = pos;
    a.Z = Z;
    a.sigma = sigma;
    a.cutoff = p->cutoff;
    a.max_sigma = p->max_sigma;
    a.info = reinterpret_cast<AtomInfo *>(p->ws + p->o_info);
    a.counts = reinterpret_cast<int32_t *>(p->ws + p->o_counts);
    a.offsets = reinterpret_cast<int32_t *>(p->ws + p->o_offsets);
    a.cursor = reinterpret_cast<int32_t *>(p->ws + p->o_cursor);
    a.list = reinterpret_cast<int32_t *>(p->ws + p->o_list);
    a.list_sorted = reinterpret_cast<int32_t *>(p->ws + p->o_lists);
    a.bpart = reinterpret_cast<double *>(p->ws + p->o_bpart);
    a.slot_of = reinterpret_cast<int32_t *>(p->ws + p->o_slot);
    a.rec = (p->fp64 || p->general) ? nullptr : reinterpret_cast<SlotAtom *>(p->ws + p->o_rec);
    a.rec64 = (!p->fp64 || p->general) ? nullptr : reinterpret_cast<SlotAtom64 *>(p->ws + p->o_rec);
    // batched plans: the matrix-core kernels take their bricks heaviest first
    // (per-brick atom counts differ several-fold between problems)
    a.order = (p->nprob > 1 && !p->general) ? reinterpret_cast<int32_t *>(p->ws + p->o_order) : nullptr;
    a.general = p->general ? 1 : 0;
    a.wide = p->wide ? 1 : 0;
    // |g|, |gd| of a c-axis factor stay below 4 max(1, max_sigma) (a few
    // images at most, |d| e^(-d^2 / 2 sigma^2) <= 0.61 sigma): scaled by
    // 2^b_exp they stay below 2^14, inside the 16-bit range
    a.b_exp = int(std::floor(std::log2(16384.0 / (4.0 * std::max(1.0, p->max_sigma)))));
    a.b_exp = std::min(14, std::max(-60, a.b_exp));
    // a prime stride that does not divide natoms permutes the atoms
    a.visit_stride = 1;
    for (int32_t pr : {1009, 1013, 1019}) {
        if (natoms % pr != 0) {
            a.visit_stride = pr;
            break;
        }
    }
    a.zeros = reinterpret_cast<const float *>(p->ws + p->o_zero);
    a.cap_pa = p->cap_pa;
    a.capacity = p->capacity;
    a.nbricks_total = p->nbricks;
    a.status = reinterpret_cast<DeviceStatus *>(p->ws + p->o_status);
    a.fp64 = p->fp64;
    a.qsum = reinterpret_cast<double *>(p->ws + p->o_qsum);
    return a;
}

hartree_status check_atoms(hartree_plan p, int32_t natoms, const double *pos, const double *Z, const double *sigma,
                           const int32_t *atom_offsets)
{
    if (!p->splat_ok) return fail(HARTREE_ERR_UNSUPPORTED, "the plan has no splat workspace");
    if (natoms < 0) return fail(HARTREE_ERR_ARG, "natoms < 0");
    if (natoms > p->max_atoms)
        return fail(HARTREE_ERR_ARG, "natoms %d exceeds the plan's max_atoms %d", natoms, p->max_atoms);
    if (natoms > 0 && (!pos || !Z || !sigma)) return fail(HARTREE_ERR_ARG, "pos, Z or sigma is NULL");
    if (p->nprob > 1) {
        if (!atom_offsets) return fail(HARTREE_ERR_ARG, "batched plans need atom_offsets");
        if (atom_offsets[0] != 0 || atom_offsets[p->nprob] != natoms)
            return fail(HARTREE_ERR_ARG, "atom_offsets must start at 0 and end at natoms");
        for (int i = 0; i < p->nprob; ++i)
            if (atom_offsets[i + 1] < atom_offsets[i]) return fail(HARTREE_ERR_ARG, "atom_offsets must not decrease");
    } else if (atom_offsets) {
        if (atom_offsets[0] != 0 || atom_offsets[1] != natoms)
            return fail(HARTREE_ERR_ARG, "atom_offsets must be {0, natoms}");
    }
    return HARTREE_OK;
}

}  // namespace

extern "C" {

hartree_status hartree_plan_create(hartree_plan *out, const double cell[9], const int32_t dims[3], int32_t precision,
                                   const hartree_plan_opts *opts)
{
    return create(out, 1, cell, dims, precision, opts);
}

hartree_status hartree_plan_create_batched(hartree_plan *out, int32_t nprob, const double *cells, const int32_t *dims,
                                           int32_t precision, const hartree_plan_opts *opts)
{
    return create(out, nprob, cells, dims, precision, opts);
}

void hartree_plan_destroy(hartree_plan plan) { delete plan; }

hartree_status hartree_plan_nprob(hartree_plan plan, int32_t *nprob)
{
    if (!plan || !nprob) return fail(HARTREE_ERR_ARG, "NULL argument");
    *nprob = plan->nprob;
    return ok();
}

hartree_status hartree_plan_grid_offset(hartree_plan plan, int32_t p, int64_t *offset)
{
    if (!plan || !offset) return fail(HARTREE_ERR_ARG, "NULL argument");
    if (p < 0 || p > plan->nprob) return fail(HARTREE_ERR_ARG, "problem index %d out of range", p);
    *offset = plan->grid_offsets[p];
    return ok();
}

hartree_status hartree_workspace_size(hartree_plan plan, size_t *bytes)
{
    if (!plan || !bytes) return fail(HARTREE_ERR_ARG, "NULL argument");
    *bytes = plan->ws_size;
    return ok();
}

hartree_status hartree_bind_workspace(hartree_plan plan, void *workspace, size_t bytes)
{
    if (!plan || !workspace) return fail(HARTREE_ERR_ARG, "NULL argument");
    if (plan->capturing) return fail(HARTREE_ERR_ARG, "cannot bind a workspace during graph capture");
    if (bytes < plan->ws_size)
        return fail(HARTREE_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu needed", bytes,
                    plan->ws_size);
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return fail(HARTREE_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    unsigned char *ws = static_cast<unsigned char *>(workspace);
    hipError_t e = hipMemcpy(ws + plan->o_desc, plan->desc.data(), sizeof(ProbDesc) * plan->nprob,
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "uploading plan descriptors");
    const size_t ntw = plan->twiddles.size() / 2;
    if (plan->fp64) {
        e = hipMemcpy(ws + plan->o_tw, plan->twiddles.data(), 16 * ntw, hipMemcpyHostToDevice);
    } else {
        std::vector<float> f(plan->twiddles.size());
        for (size_t i = 0; i < f.size(); ++i) f[i] = float(plan->twiddles[i]);
        e = hipMemcpy(ws + plan->o_tw, f.data(), 8 * ntw, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return hip_fail(e, "uploading twiddles");
    DeviceStatus st;
    std::memset(&st, 0, sizeof(st));
    e = hipMemcpy(ws + plan->o_status, &st, sizeof(st), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "clearing the status word");
    const unsigned char zero[256] = {};
    e = hipMemcpy(ws + plan->o_zero, zero, sizeof(zero), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "clearing the zero block");
    if (!plan->side_ready) {
        // side streams for the launch groups of batched passes and the
        // backward chain of hartree_solve_backward (on the device current
        // now, the workspace's); without them that work runs in order on the
        // caller's stream
        bool okay = true;
        for (int i = 0; i < hartree_plan_s::kSide && okay; ++i)
            okay = hipStreamCreateWithFlags(&plan->side[i], hipStreamNonBlocking) == hipSuccess &&
                   hipEventCreateWithFlags(&plan->join_ev[i], hipEventDisableTiming) == hipSuccess;
        okay = okay && hipStreamCreateWithFlags(&plan->chain_side, hipStreamNonBlocking) == hipSuccess;
        for (hipEvent_t *q : {&plan->fork_ev, &plan->chain_fork, &plan->chain_join})
            okay = okay && hipEventCreateWithFlags(q, hipEventDisableTiming) == hipSuccess;
        if (okay) plan->side_ready = true;
        else plan->drop_side();
    }
    if (plan->splat_ok) {
        // binning keeps its brick counters cleared from one call to the next
        e = hipMemset(ws + plan->o_counts, 0, 4 * size_t(plan->nbricks + 1));
        if (e == hipSuccess) e = hipMemset(ws + plan->o_cursor, 0, 4 * size_t(plan->nbricks + 1));
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "clearing the brick counters");
    }
    plan->ws = ws;
    return ok();
}

namespace {
// P1..P5 of the solve on stream s (a.in = rho, a.out = v), with the E_H
// finalize after P3
hartree_status solve_chain(hartree_plan plan, PassArgs a, double *e_h, hipStream_t s)
{
    hipError_t e;
    if ((e = run_group(plan, plan->lr2c, PASS_R2C_FWD, a, s)) != hipSuccess) return hip_fail(e, "P1");
    if ((e = run_group(plan, plan->lb, PASS_B_FWD, a, s)) != hipSuccess) return hip_fail(e, "P2");
    if ((e = run_group(plan, plan->la, e_h ? PASS_A_FULL : PASS_A_NOENERGY, a, s)) != hipSuccess)
        return hip_fail(e, "P3");
    // the E_H sum in order on s: beside P4 and P5 on a side stream, the fork
    // and the join cost more (a gap before P4 and one after P5) than the
    // short kernel does in order
    if (e_h && (e = timed(plan, HARTREE_K_FINALIZE, s, [&]() {
                    return run_finalize(a.desc, a.partials, e_h, plan->nprob, s);
                })) != hipSuccess)
        return hip_fail(e, "E_H finalize");
    if ((e = run_group(plan, plan->lb, PASS_B_INV, a, s)) != hipSuccess) return hip_fail(e, "P4");
    if ((e = run_group(plan, plan->lr2c, PASS_C2R, a, s)) != hipSuccess) return hip_fail(e, "P5");
    return ok();
}


}  // namespace

hartree_status hartree_solve(hartree_plan plan, const void *rho, void *v, double *e_h, void *stream)
{
    hartree_status st = check_ws(plan);
    if (st != HARTREE_OK) return st;
    if (!rho || !v) return fail(HARTREE_ERR_ARG, "rho or v is NULL");
    if (rho == v) return fail(HARTREE_ERR_ARG, "v may not alias rho");
    PassArgs a = base_args(plan);
    a.in = rho;
    a.out = v;
    return solve_chain(plan, a, e_h, static_cast<hipStream_t>(stream));
}

hartree_status hartree_energy(hartree_plan plan, const void *rho, double *e_h, void *stream)
{
    hartree_status st = check_ws(plan);
    if (st != HARTREE_OK) return st;
    if (!rho || !e_h) return fail(HARTREE_ERR_ARG, "rho or e_h is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    PassArgs a = base_args(plan);
    a.in = rho;
    hipError_t e;
    if ((e = run_group(plan, plan->lr2c, PASS_R2C_FWD, a, s)) != hipSuccess) return hip_fail(e, "P1");
    if ((e = run_group(plan, plan->lb, PASS_B_FWD, a, s)) != hipSuccess) return hip_fail(e, "P2");
    if ((e = run_group(plan, plan->la, PASS_A_ENERGY, a, s)) != hipSuccess) return hip_fail(e, "P3");
    if ((e = timed(plan, HARTREE_K_FINALIZE, s, [&]() { return run_finalize(a.desc, a.partials, e_h, plan->nprob, s); })) !=
        hipSuccess)
        return hip_fail(e, "E_H finalize");
    return ok();
}

namespace {
// P1..P5 of the backward on stream s (a.in = grad_v, a.in2 = rho, a.grad_e,
// a.out = grad_rho)
hartree_status backward_chain(hartree_plan plan, PassArgs a, hipStream_t s)
{
    hipError_t e;
    if (!a.in && !a.grad_e) {  // no upstream gradient: the result is zero
        if ((e = run_zero(a.out, size_t(plan->grid_total) * (plan->fp64 ? 8 : 4), s)) != hipSuccess)
            return hip_fail(e, "zeroing grad_rho");
        return ok();
    }
    if ((e = run_group(plan, plan->lr2c, PASS_R2C_BWD, a, s)) != hipSuccess) return hip_fail(e, "P1");
    if ((e = run_group(plan, plan->lb, PASS_B_FWD, a, s)) != hipSuccess) return hip_fail(e, "P2");
    if ((e = run_group(plan, plan->la, PASS_A_NOENERGY, a, s)) != hipSuccess) return hip_fail(e, "P3");
    if ((e = run_group(plan, plan->lb, PASS_B_INV, a, s)) != hipSuccess) return hip_fail(e, "P4");
    if ((e = run_group(plan, plan->lr2c, PASS_C2R, a, s)) != hipSuccess) return hip_fail(e, "P5");
    return ok();
}

hartree_status check_backward_args(const void *grad_v, const double *grad_e, const void *rho, const void *grad_rho)
{
    if (!grad_rho) return fail(HARTREE_ERR_ARG, "grad_rho is NULL");
    if (grad_e && !rho) return fail(HARTREE_ERR_ARG, "rho is needed when grad_e is given");
    if (grad_rho == grad_v || grad_rho == rho) return fail(HARTREE_ERR_ARG, "grad_rho may not alias an input");
    return ok();
}
}  // namespace

hartree_status hartree_backward(hartree_plan plan, const void *grad_v, const double *grad_e, const void *rho,
                                void *grad_rho, void *stream)
{
    hartree_status st = check_ws(plan);
    if (st != HARTREE_OK) return st;
    if ((st = check_backward_args(grad_v, grad_e, rho, grad_rho)) != HARTREE_OK) return st;
    PassArgs a = base_args(plan);
    a.in = grad_v;
    a.in2 = rho;
    a.grad_e = grad_e;
    a.out = grad_rho;
    return backward_chain(plan, a, static_cast<hipStream_t>(stream));
}

// the last-level cache (MI355X: 256 MiB of Infinity Cache) that two spectra
// side by side must fit for hartree_solve_backward to overlap its chains
constexpr size_t kOverlapCacheBytes = size_t(256) << 20;

hartree_status hartree_solve_backward(hartree_plan plan, const void *rho, void *v, double *e_h, const void *grad_v,
                                      const double *grad_e, void *grad_rho, void *stream)
{
    hartree_status st = check_ws(plan);
    if (st != HARTREE_OK) return st;
    if (!rho || !v) return fail(HARTREE_ERR_ARG, "rho or v is NULL");
    if (rho == v) return fail(HARTREE_ERR_ARG, "v may not alias rho");
    if ((st = check_backward_args(grad_v, grad_e, rho, grad_rho)) != HARTREE_OK) return st;
    if (v == grad_v || v == grad_rho)
        return fail(HARTREE_ERR_ARG, "v may not alias grad_v or grad_rho (the two chains run concurrently)");
    hipStream_t s = static_cast<hipStream_t>(stream);
    PassArgs a = base_args(plan);
    a.in = rho;
    a.out = v;
    PassArgs b = base_args(plan);
    b.spec = plan->ws + plan->o_spec2;  // the backward chain's own spectrum
    b.in = grad_v;
    b.in2 = rho;
    b.grad_e = grad_e;
    b.out = grad_rho;
    // The chains run side by side when their two spectra fit the last-level
    // cache together, and every pass is one launch group (single plans;
    // batched plans whose problems all take multi-plan launches), so that the
    // backward chain forks no side streams of its own.  Otherwise, or without
    // the plan's streams, in order on the caller's stream: a spectrum that
    // fits the cache alone stays there from one pass to the next, which two
    // chains side by side would give up.
    const bool single_groups = plan->lr2c.size() == 1 && plan->lb.size() == 1 && plan->la.size() == 1;
    const size_t spec_bytes = size_t(plan->spec_count) * (plan->fp64 ? 16 : 8);
    if (!plan->side_ready || !single_groups || 2 * spec_bytes > kOverlapCacheBytes) {
        // in order, on the one spectrum (the cache still holds it)
        if ((st = solve_chain(plan, a, e_h, s)) != HARTREE_OK) return st;
        b.spec = a.spec;
        return backward_chain(plan, b, s);
    }
    // The forward chain (the shorter one: its P1 reads one grid, the
    // backward's two) forks onto the plan's stream after the work already on
    // s (rho's producer); the backward chain stays on s, so that the join
    // before the caller's next work (the adjoint) finds the forward chain
    // already done.  The join comes also after an error, so that no capture
    // keeps an open branch.
    hipError_t e = hipEventRecord(plan->chain_fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(plan->chain_side, plan->chain_fork, 0);
    if (e != hipSuccess) return hip_fail(e, "forking the forward chain");
    const hartree_status sf = solve_chain(plan, a, e_h, plan->chain_side);
    const hartree_status sb = sf == HARTREE_OK ? backward_chain(plan, b, s) : sf;
    e = hipEventRecord(plan->chain_join, plan->chain_side);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, plan->chain_join, 0);
    if (e != hipSuccess) return hip_fail(e, "joining the forward chain");
    if (sf != HARTREE_OK) return sf;
    return sb;
}

hartree_status hartree_atoms_bind(hartree_plan plan, int32_t natoms, const double *pos, const double *Z,
                                  const double *sigma, const int32_t *atom_offsets, uint64_t *token, void *stream)
{
    hartree_status st = check_ws(plan);
    if (st != HARTREE_OK) return st;
    if ((st = check_atoms(plan, natoms, pos, Z, sigma, atom_offsets)) != HARTREE_OK) return st;
    SplatArgs a = splat_args(plan, natoms, pos, Z, sigma, atom_offsets);
    hipStream_t s = static_cast<hipStream_t>(stream);
    plan->bound = false;
    hipError_t e = timed(plan, HARTREE_K_BIN, s, [&]() { return run_bin(a, s); });
    if (e != hipSuccess) return hip_fail(e, "atom binning");
    plan->bound = true;
    plan->bind_token += 1;
    plan->bound_natoms = natoms;
    plan->bound_pos = pos;
    plan->bound_Z = Z;
    plan->bound_sigma = sigma;
    plan->bound_offsets.assign(a.atom_off, a.atom_off + plan->nprob + 1);
    if (token) *token = plan->bind_token;
    return ok();
}

namespace {
hartree_status bound_args(hartree_plan plan, uint64_t token, SplatArgs &a)
{
    hartree_status st = check_ws(plan);
    if (st != HARTREE_OK) return st;
    if (!plan->bound || token != plan->bind_token)
        return fail(HARTREE_ERR_ARG, "atom binding %llu is not current (current %llu)", (unsigned long long)token,
                    (unsigned long long)plan->bind_token);
    a = splat_args(plan, plan->bound_natoms, plan->bound_pos, plan->bound_Z, plan->bound_sigma,
                   plan->nprob > 1 ? plan->bound_offsets.data() : nullptr);
    return HARTREE_OK;
}
}  // namespace

hartree_status hartree_splat_bound(hartree_plan plan, uint64_t token, void *rho_out, int32_t subtract_background,
                                   void *stream)
{
    SplatArgs a;
    hartree_status st = bound_args(plan, token, a);
    if (st != HARTREE_OK) return st;
    if (!rho_out) return fail(HARTREE_ERR_ARG, "rho_out is NULL");
    a.rho = rho_out;
    a.subtract_background = subtract_background ? 1 : 0;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = timed(plan, HARTREE_K_SPLAT, s, [&]() { return run_gather(a, s); });
    if (e != hipSuccess) return hip_fail(e, "splat");
    return ok();
}

hartree_status hartree_splat_adjoint_bound(hartree_plan plan, uint64_t token, const void *grad_rho, double *grad_pos,
                                           void *stream)
{
    SplatArgs a;
    hartree_status st = bound_args(plan, token, a);
    if (st != HARTREE_OK) return st;
    if (!grad_rho || (a.natoms > 0 && !grad_pos)) return fail(HARTREE_ERR_ARG, "grad_rho or grad_pos is NULL");
    a.grad_rho = grad_rho;
    a.grad_pos = grad_pos;
    // 16-byte row loads where a problem's rows are whole, aligned vectors:
    // 1 when that holds for every problem, 2 when only some (the kernels
    // check each problem's row length and offset), 0 for an unaligned grid
    a.grad_rows_vec16 = 0;
    if (reinterpret_cast<uintptr_t>(grad_rho) % 16 == 0) {
        const int per = plan->fp64 ? 2 : 4;  // elements per 16-byte vector
        a.grad_rows_vec16 = 1;
        for (const ProbDesc &d : plan->desc)
            if (d.dims[2] % per != 0 || d.grid_off % per != 0) a.grad_rows_vec16 = 2;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = timed(plan, HARTREE_K_ADJOINT, s, [&]() { return run_adjoint(a, s); });
    if (e != hipSuccess) return hip_fail(e, "splat adjoint");
    e = timed(plan, HARTREE_K_ADJOINT_FINAL, s, [&]() { return run_adjoint_final(a, s); });
    if (e != hipSuccess) return hip_fail(e, "splat adjoint reduction");
    return ok();
}

hartree_status hartree_splat(hartree_plan plan, int32_t natoms, const double *pos, const double *Z,
                             const double *sigma, const int32_t *atom_offsets, void *rho_out,
                             int32_t subtract_background, void *stream)
{
    if (!rho_out) return fail(HARTREE_ERR_ARG, "rho_out is NULL");
    uint64_t token = 0;
    hartree_status st = hartree_atoms_bind(plan, natoms, pos, Z, sigma, atom_offsets, &token, stream);
    if (st != HARTREE_OK) return st;
    return hartree_splat_bound(plan, token, rho_out, subtract_background, stream);
}

hartree_status hartree_splat_adjoint(hartree_plan plan, int32_t natoms, const double *pos, const double *Z,
                                     const double *sigma, const int32_t *atom_offsets, const void *grad_rho,
                                     double *grad_pos, void *stream)
{
    if (!grad_rho || (natoms > 0 && !grad_pos)) return fail(HARTREE_ERR_ARG, "grad_rho or grad_pos is NULL");
    uint64_t token = 0;
    hartree_status st = hartree_atoms_bind(plan, natoms, pos, Z, sigma, atom_offsets, &token, stream);
    if (st != HARTREE_OK) return st;
    return hartree_splat_adjoint_bound(plan, token, grad_rho, grad_pos, stream);
}

hartree_status hartree_atoms_pairs(hartree_plan plan, int64_t *pairs, void *stream)
{
    hartree_status st = check_ws(plan);
    if (st != HARTREE_OK) return st;
    if (plan->capturing) return fail(HARTREE_ERR_ARG, "the binding size cannot be read during graph capture");
    if (!pairs) return fail(HARTREE_ERR_ARG, "pairs is NULL");
    if (!plan->splat_ok) {
        *pairs = 0;
        return ok();
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    int32_t v = 0;
    hipError_t e = hipMemcpyAsync(&v, plan->ws + plan->o_offsets + 4 * size_t(plan->nbricks), 4,
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "reading the binding size");
    *pairs = v;
    return ok();
}

hartree_status hartree_device_status(hartree_plan plan, uint32_t *bits, void *stream)
{
    hartree_status st = check_ws(plan);
    if (st != HARTREE_OK) return st;
    if (plan->capturing) return fail(HARTREE_ERR_ARG, "the status word cannot be read during graph capture");
    if (!bits) return fail(HARTREE_ERR_ARG, "bits is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint32_t v = 0;
    hipError_t e = hipMemcpyAsync(&v, plan->ws + plan->o_status, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "reading the status word");
    const uint32_t zero = 0;
    e = hipMemcpy(plan->ws + plan->o_status, &zero, 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "clearing the status word");
    *bits = v;
    return ok();
}

hartree_status hartree_profile_begin(hartree_plan plan)
{
    if (!plan) return fail(HARTREE_ERR_ARG, "plan is NULL");
    plan->recs.clear();
    plan->pool_used = 0;
    plan->prof = true;
    return ok();
}

hartree_status hartree_profile_end(hartree_plan plan, double *total_ms, int64_t *launches)
{
    if (!plan || !total_ms || !launches) return fail(HARTREE_ERR_ARG, "NULL argument");
    plan->prof = false;
    for (int i = 0; i < HARTREE_K_COUNT; ++i) {
        total_ms[i] = 0.0;
        launches[i] = 0;
    }
    if (!plan->recs.empty()) {
        hipError_t e = hipEventSynchronize(plan->recs.back().b);
        if (e != hipSuccess) return hip_fail(e, "waiting for the profiling events");
    }
    for (const auto &r : plan->recs) {
        float ms = 0.0f;
        hipError_t e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) return hip_fail(e, "reading a profiling event");
        total_ms[r.id] += ms;
        launches[r.id] += 1;
    }
    plan->recs.clear();
    plan->pool_used = 0;
    return ok();
}

hartree_status hartree_graph_begin(hartree_plan plan, void *stream)
{
    hartree_status st = check_ws(plan);
    if (st != HARTREE_OK) return st;
    if (plan->capturing) return fail(HARTREE_ERR_ARG, "a capture is already open on this plan");
    if (!stream) return fail(HARTREE_ERR_ARG, "capture needs a created stream, not the default stream");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "beginning stream capture");
    plan->capturing = true;
    plan->cap_stream = s;
    return ok();
}

hartree_status hartree_graph_end(hartree_plan plan, void *stream)
{
    if (!plan) return fail(HARTREE_ERR_ARG, "plan is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!plan->capturing || s != plan->cap_stream)
        return fail(HARTREE_ERR_ARG, "no capture open on this plan and stream");
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    plan->capturing = false;
    plan->cap_stream = nullptr;
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(e, "ending stream capture");
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(e, "instantiating the captured graph");
    }
    plan->drop_graph();
    plan->graph = g;
    plan->graph_exec = x;
    return ok();
}

hartree_status hartree_graph_launch(hartree_plan plan, void *stream)
{
    if (!plan) return fail(HARTREE_ERR_ARG, "plan is NULL");
    if (!plan->graph_exec) return fail(HARTREE_ERR_ARG, "no graph captured on this plan");
    if (plan->capturing) return fail(HARTREE_ERR_ARG, "a capture is open on this plan");
    hipError_t e = hipGraphLaunch(plan->graph_exec, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "launching the captured graph");
    return ok();
}

namespace {

// largest dynamic LDS a workgroup may opt in to on the current device
size_t lds_cap()
{
    static size_t cap = 0;
    if (cap == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeSharedMemPerBlockOptin, dev) == hipSuccess && v > 0)
            cap = size_t(v);
        else
            cap = 65536;
    }
    return cap;
}

// radices of an axis choice for length n along axis x (plan < 0: the
// default factorization on the run-time radix kernel); false if it does not
// apply.  The pad applies to the strided axes a and b only.
bool choice_radices(hartree_plan p, int x, int n, int plan, int p_log2, int pad, std::vector<int> &r)
{
    r.clear();
    if (plan >= 0) {
        if (plan >= plan_table_size()) return false;
        int rad[4];
        const int ns = plan_table_row(plan, rad);
        long prod = 1;
        for (int s = 0; s < ns; ++s) {
            r.push_back(rad[s]);
            prod *= rad[s];
        }
        if (prod != n) return false;
    } else if (!factorize(n, p->fp64, r)) {
        return false;
    }
    if (p_log2 < 0 || p_log2 > 8) return false;
    if (pad < 0 || pad > 3 || (x == 2 && pad != 0)) return false;
    const int tpp = pass_min_tpp(p->fp64, n, r.data(), int(r.size()));
    if ((256 >> p_log2) < tpp) return false;  // 256 threads per pass workgroup
    return pass_tile_lds(p->fp64, n, p_log2, pad) <= lds_cap();
}

void set_axis(ProbDesc &d, int x, const std::vector<int> &r)
{
    AxisPlan &ap = d.ax[x];
    const int n = ap.n;
    ap.nstages = int(r.size());
    int ns = 1;
    for (int s = 0; s < kMaxStages; ++s) {
        ap.radix[s] = s < ap.nstages ? r[s] : 0;
        ap.twstride[s] = 0;
        ap.ns[s] = make_fastdiv(1u);
    }
    for (int s = 0; s < ap.nstages; ++s) {
        ap.ns[s] = make_fastdiv(uint32_t(ns));
        ap.twstride[s] = n / (ns * r[s]);
        ns *= r[s];
    }
}

hartree_status upload_desc(hartree_plan p)
{
    if (!p->ws) return HARTREE_OK;
    hipError_t e = hipMemcpy(p->ws + p->o_desc, p->desc.data(), sizeof(ProbDesc) * p->nprob, hipMemcpyHostToDevice);
    return e == hipSuccess ? HARTREE_OK : hip_fail(e, "uploading problem descriptors");
}

// apply per-(problem, axis) choices (plan, p_log2, pad) after validating all
hartree_status apply_config(hartree_plan p, const int32_t *cfg)
{
    std::vector<std::vector<int>> rad(3 * p->nprob);
    for (int q = 0; q < p->nprob; ++q)
        for (int x = 0; x < 3; ++x) {
            const int32_t *c = cfg + 3 * (3 * q + x);
            if (!choice_radices(p, x, p->desc[q].dims[x], c[0], c[1], c[2], rad[3 * q + x]))
                return fail(HARTREE_ERR_ARG,
                            "problem %d axis %d: plan %d with 2^%d pencils and pad %d does not apply to length %d", q,
                            x, c[0], c[1], c[2], p->desc[q].dims[x]);
        }
    for (int q = 0; q < p->nprob; ++q)
        for (int x = 0; x < 3; ++x) {
            const int32_t *c = cfg + 3 * (3 * q + x);
            set_axis(p->desc[q], x, rad[3 * q + x]);
            p->cfg[3 * q + x] = {c[0], c[1], c[2]};
        }
    rebuild_launches(p);
    return upload_desc(p);
}

void get_config(hartree_plan p, std::vector<int32_t> &cfg)
{
    cfg.resize(9 * size_t(p->nprob));
    for (size_t i = 0; i < p->cfg.size(); ++i) {
        cfg[3 * i] = p->cfg[i].plan;
        cfg[3 * i + 1] = p->cfg[i].p_log2;
        cfg[3 * i + 2] = p->cfg[i].pad;
    }
}

// enqueue the passes along axis x (both directions) once
hipError_t run_axis(hartree_plan p, int x, void *grid, hipStream_t s)
{
    PassArgs a = base_args(p);
    a.in = grid;
    a.out = grid;
    hipError_t e;
    if (x == 2) {
        if ((e = run_group(p, p->lr2c, PASS_R2C_FWD, a, s)) != hipSuccess) return e;
        return run_group(p, p->lr2c, PASS_C2R, a, s);
    }
    if (x == 1) {
        if ((e = run_group(p, p->lb, PASS_B_FWD, a, s)) != hipSuccess) return e;
        return run_group(p, p->lb, PASS_B_INV, a, s);
    }
    return run_group(p, p->la, PASS_A_FULL, a, s);
}

}  // namespace

hartree_status hartree_plan_get_config(hartree_plan plan, int32_t *cfg)
{
    if (!plan || !cfg) return fail(HARTREE_ERR_ARG, "NULL argument");
    std::vector<int32_t> c;
    get_config(plan, c);
    std::copy(c.begin(), c.end(), cfg);
    return ok();
}

hartree_status hartree_plan_set_config(hartree_plan plan, const int32_t *cfg)
{
    if (!plan || !cfg) return fail(HARTREE_ERR_ARG, "NULL argument");
    if (plan->capturing) return fail(HARTREE_ERR_ARG, "cannot change the plan during graph capture");
    hartree_status st = apply_config(plan, cfg);
    return st == HARTREE_OK ? ok() : st;
}

hartree_status hartree_plan_tune(hartree_plan plan, void *grid, int32_t reps, void *stream)
{
    hartree_status st = check_ws(plan);
    if (st != HARTREE_OK) return st;
    if (!grid) return fail(HARTREE_ERR_ARG, "the scratch grid is NULL");
    if (reps < 1 || reps > 1000) return fail(HARTREE_ERR_ARG, "reps must be in [1, 1000]");
    if (plan->capturing || plan->prof) return fail(HARTREE_ERR_ARG, "cannot tune during capture or profiling");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t ev[2] = {nullptr, nullptr};
    if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess) {
        if (ev[0]) (void)hipEventDestroy(ev[0]);
        return fail(HARTREE_ERR_HIP, "creating timing events");
    }
    std::vector<int32_t> cfg;
    get_config(plan, cfg);
    hartree_status result = HARTREE_OK;
    // time the passes along axis x under configuration c (reps runs after a
    // warm-up); false when c does not apply
    auto time_axis = [&](int x, const std::vector<int32_t> &c, float &ms) -> bool {
        ms = 0.0f;
        if (apply_config(plan, c.data()) != HARTREE_OK) return false;
        hipError_t e = run_axis(plan, x, grid, s);  // warm-up (and attribute opt-in)
        if (e == hipSuccess) e = hipEventRecord(ev[0], s);
        for (int i = 0; i < reps && e == hipSuccess; ++i) e = run_axis(plan, x, grid, s);
        if (e == hipSuccess) e = hipEventRecord(ev[1], s);
        if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
        if (e != hipSuccess) {
            result = hip_fail(e, "timing a pass candidate");
            return false;
        }
        return true;
    };
    // one key per (axis, length): every problem with that length takes the choice
    for (int x = 2; x >= 0 && result == HARTREE_OK; --x) {
        std::vector<int> lengths;
        for (int q = 0; q < plan->nprob; ++q)
            if (std::find(lengths.begin(), lengths.end(), plan->desc[q].dims[x]) == lengths.end())
                lengths.push_back(plan->desc[q].dims[x]);
        for (int n : lengths) {
            struct Cand {
                int id, lp, pad;
            };
            std::vector<Cand> cand;
            std::vector<int> r;
            for (int id = -1; id < plan_table_size(); ++id)
                for (int lp = 0; lp <= 6; ++lp)
                    for (int pad = 0; pad <= (x == 2 ? 0 : 2); ++pad)
                        if (choice_radices(plan, x, n, id, lp, pad, r) &&
                            (id >= 0 || find_plan(r.data(), int(r.size())) < 0))
                            cand.push_back({id, lp, pad});
            float best = 0.0f;
            std::vector<int32_t> best_cfg = cfg;
            for (const auto &c : cand) {
                std::vector<int32_t> trial = cfg;
                for (int q = 0; q < plan->nprob; ++q)
                    if (plan->desc[q].dims[x] == n) {
                        trial[3 * (3 * q + x)] = c.id;
                        trial[3 * (3 * q + x) + 1] = c.lp;
                        trial[3 * (3 * q + x) + 2] = c.pad;
                    }
                float ms = 0.0f;
                if (!time_axis(x, trial, ms)) {
                    if (result != HARTREE_OK) break;
                    continue;
                }
                if (best == 0.0f || ms < best) {
                    best = ms;
                    best_cfg = trial;
                }
            }
            if (result != HARTREE_OK) break;
            cfg = best_cfg;
        }
        // batched FP32 plans: the axis as one multi-plan launch per pass
        // (every length on its compiled plan at the multi tile width), kept
        // when it times faster than the per-length choices
        if (result == HARTREE_OK && plan->nprob > 1 && !plan->fp64) {
            float ms_best = 0.0f;
            if (!time_axis(x, cfg, ms_best)) ms_best = 0.0f;
            for (int lp : {multi_log_p(x, 0), multi_log_p(x, 1), kMultiAutoLog}) {
                if (result != HARTREE_OK || ms_best == 0.0f) break;
                std::vector<int32_t> trial = cfg;
                bool whole = true;
                for (int q = 0; q < plan->nprob && whole; ++q) {
                    const int n = plan->desc[q].dims[x];
                    int id = -1;
                    for (int i = 0; i < kMultiPlans && id < 0; ++i) {
                        int rad[4];
                        const int ns = plan_table_row(multi_plans(x)[i], rad);
                        long prod = 1;
                        for (int k = 0; k < ns; ++k) prod *= rad[k];
                        if (prod == n) id = multi_plans(x)[i];
                    }
                    whole = id >= 0;
                    int l2 = lp;
                    if (lp == kMultiAutoLog)
                        for (l2 = 0; (1 << l2) < multi_auto_p(n, x); ++l2) {
                        }
                    trial[3 * (3 * q + x)] = id;
                    trial[3 * (3 * q + x) + 1] = l2;
                    trial[3 * (3 * q + x) + 2] = 0;
                }
                float ms = 0.0f;
                if (whole && time_axis(x, trial, ms) && ms < ms_best) {
                    ms_best = ms;
                    cfg = trial;
                }
            }
        }
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    hartree_status st2 = apply_config(plan, cfg.data());
    if (result != HARTREE_OK) return result;
    return st2 == HARTREE_OK ? ok() : st2;
}

}  // extern "C"

// ------------------------------------------------------ no-allocation solve
// The device scratch of hartree_solve_noalloc: one copy of this array per GPU
// (created with the code object, held until the process ends), laid out like
// the first part of a plan's workspace (status word, zero block, problem
// descriptors, twiddles, half spectrum, E_H partials).  Host code never uses
// the array's name as an address: each GPU's copy is found with
// hipGetSymbolAddress (noalloc_scratch below), and only that pointer is
// passed to kernels.
static __device__ __align__(256) unsigned char scratch[HARTREE_NOALLOC_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

// device address of the current device's scratch, looked up once per device
hipError_t noalloc_scratch(unsigned char **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr || reinterpret_cast<uintptr_t>(ptr) % 256 != 0) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = static_cast<unsigned char *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// cos and sin of 2 pi t / n, the angle reduced to the first octant in
// integer arithmetic as on the host (FP64 device cos / sin)
__device__ void unit_root_dev(int t, int n, double &c, double &s)
{
    const int u = 4 * t;  // t < n <= 4096
    const int q = u / n;
    int r = u - q * n;
    bool swap = false;
    if (2 * r > n) {
        r = n - r;
        swap = true;
    }
    const double th = 1.5707963267948966192313216916397514 * double(r) / double(n);
    double cc = cos(th), ss = sin(th);
    if (swap) {
        const double tmp = cc;
        cc = ss;
        ss = tmp;
    }
    switch (q) {
    case 0: c = cc; s = ss; break;
    case 1: c = -ss; s = cc; break;
    case 2: c = -cc; s = -ss; break;
    default: c = ss; s = -cc; break;
    }
}

// One problem's descriptor (thread 0 of block 0) and the twiddle tables of its
// three axes, W_n^t = exp(-2 pi i t / n) in the plan's precision, into the
// scratch.  Problems sharing a length write the same values to the same table.
template <typename T>
__global__ __launch_bounds__(256) void k_noalloc_setup(ProbDesc d, ProbDesc *desc_out, Cx<T> *tw)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) *desc_out = d;
    for (int x = 0; x < 3; ++x) {
        const int n = d.ax[x].n;
        if (t < n) {
            double c, s;
            unit_root_dev(t, n, c, s);
            tw[d.ax[x].tw_off + t] = Cx<T>{T(c), T(-s)};
        }
    }
}

// the launch groups of one pass, in order on one stream
hipError_t run_group_serial(hartree_plan p, const std::vector<Launch> &groups, PassKind kind, PassArgs a,
                            hipStream_t s)
{
    for (const Launch &l : groups) {
        a.tl = l.tl;
        a.col_stride = l.col_stride;
        hipError_t e = run_pass(p->fp64, kind, l.plan, l.p_log2, l.pad, l.maxn, l.tl.total, s, a);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

hartree_status hartree_solve_noalloc(hartree_plan plan, const void *rho, void *v, double *e_h, void *stream)
{
    if (!plan) return fail(HARTREE_ERR_ARG, "plan is NULL");
    if (!rho || !v) return fail(HARTREE_ERR_ARG, "rho or v is NULL");
    if (rho == v) return fail(HARTREE_ERR_ARG, "v may not alias rho");
    // the workspace up to the E_H partials: what the solve uses
    const size_t need = plan->o_qsum;
    if (need > size_t(HARTREE_NOALLOC_BYTES))
        return fail(HARTREE_ERR_WORKSPACE,
                    "the plan needs %zu bytes of scratch; hartree_solve_noalloc holds %zu (HARTREE_NOALLOC_BYTES): "
                    "use hartree_solve with a bound workspace",
                    need, size_t(HARTREE_NOALLOC_BYTES));
    unsigned char *ws = nullptr;
    hipError_t e = noalloc_scratch(&ws);
    if (e != hipSuccess) return hip_fail(e, "locating the device scratch");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int maxn = 1;
    for (const ProbDesc &d : plan->desc)
        for (int x = 0; x < 3; ++x) maxn = std::max(maxn, d.ax[x].n);
    const int blocks = (maxn + 255) / 256;
    for (int q = 0; q < plan->nprob; ++q) {
        ProbDesc *dst = reinterpret_cast<ProbDesc *>(ws + plan->o_desc) + q;
        if (plan->fp64)
            hipLaunchKernelGGL(k_noalloc_setup<double>, dim3(blocks), dim3(256), 0, s, plan->desc[q], dst,
                               reinterpret_cast<Cx<double> *>(ws + plan->o_tw));
        else
            hipLaunchKernelGGL(k_noalloc_setup<float>, dim3(blocks), dim3(256), 0, s, plan->desc[q], dst,
                               reinterpret_cast<Cx<float> *>(ws + plan->o_tw));
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "writing the plan into the device scratch");
    }
    PassArgs a = base_args_at(plan, ws);
    a.in = rho;
    a.out = v;
    if ((e = run_group_serial(plan, plan->lr2c, PASS_R2C_FWD, a, s)) != hipSuccess) return hip_fail(e, "P1");
    if ((e = run_group_serial(plan, plan->lb, PASS_B_FWD, a, s)) != hipSuccess) return hip_fail(e, "P2");
    if ((e = run_group_serial(plan, plan->la, e_h ? PASS_A_FULL : PASS_A_NOENERGY, a, s)) != hipSuccess)
        return hip_fail(e, "P3");
    if (e_h && (e = run_finalize(a.desc, a.partials, e_h, plan->nprob, s)) != hipSuccess)
        return hip_fail(e, "E_H finalize");
    if ((e = run_group_serial(plan, plan->lb, PASS_B_INV, a, s)) != hipSuccess) return hip_fail(e, "P4");
    if ((e = run_group_serial(plan, plan->lr2c, PASS_C2R, a, s)) != hipSuccess) return hip_fail(e, "P5");
    return ok();
}

hartree_status hartree_atom_partition(int32_t natoms, const double *pos, const double *weights, int32_t nparts,
                                      int32_t *order, int32_t *part, int32_t *part_start)
{
    const char *err = bisect_atoms(natoms, pos, weights, nparts, order, part, part_start);
    if (err) return fail(HARTREE_ERR_ARG, "%s", err);
    return ok();
}

const char *hartree_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
