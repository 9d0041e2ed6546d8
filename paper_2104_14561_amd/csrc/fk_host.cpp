// fk_host.cpp -- host runtime of the C ABI declared in include/fkexit.h:
// validation, the library's own Gauss-Hermite rule, plan tables, workspace
// carving, the backward step loop (optionally captured once in a HIP graph and
// replayed), export hooks and the checkpointed adjoint schedule.
#include "fkexit.h"
#include "fk_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

// Node classification repeats the kernels' exit comparisons; no contraction.
#pragma clang fp contract(off)

namespace {

thread_local std::string g_err;

fk_status fail(fk_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define FK_HIP(call)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(FK_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));      \
    } while (0)

constexpr int kBlock = 256;
constexpr size_t kAlign = 256;
constexpr int kProbeCkpt = 32;   // checkpoint interval of the precision probe's adjoints

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int group_of(int qs)
{
    int g = 1;
    while (g < qs) g <<= 1;
    return g;
}

// ---------------------------------------------------------------------------
// Gauss-Hermite rule: nodes are the zeros of the degree-q Hermite polynomial,
// found as the eigenvalues of the symmetric tridiagonal Jacobi matrix
// (zero diagonal, off-diagonal sqrt(k/2)) by Sturm-sequence bisection in long
// double, then polished by Newton's method on the orthonormal recurrence
//   p_{-1} = 0, p_0 = pi^{-1/4}, p_{k+1} = x sqrt(2/(k+1)) p_k - sqrt(k/(k+1)) p_{k-1},
//   p_q'(x) = sqrt(2 q) p_{q-1}(x).
// Weights are the Christoffel numbers 1 / sum_{k<q} p_k(x)^2 divided by
// sqrt(pi), so they sum to one (density pi^{-1/2} e^{-xi^2}).
// ---------------------------------------------------------------------------
using ld = long double;

int sturm_count(int q, ld x)
{
    // number of eigenvalues of the Jacobi matrix below x
    int cnt = 0;
    ld d = -x;                       // leading principal minors ratio
    if (d < 0) cnt++;
    for (int k = 1; k < q; ++k) {
        ld b2 = (ld)k / 2.0L;
        if (d == 0) d = 1e-300L;
        d = -x - b2 / d;
        if (d < 0) cnt++;
    }
    return cnt;
}

void hermite_orthonormal(int q, ld x, ld *pq, ld *pq1, ld *sumsq)
{
    ld pm1 = 0.0L, p = powl(acosl(-1.0L), -0.25L);
    ld s = p * p;
    for (int k = 0; k < q - 1; ++k) {
        ld pn = x * sqrtl(2.0L / (k + 1)) * p - sqrtl((ld)k / (k + 1)) * pm1;
        pm1 = p;
        p = pn;
        s += p * p;
    }
    // p = p_{q-1}, pm1 = p_{q-2}; one more step for p_q
    ld pqv = x * sqrtl(2.0L / q) * p - sqrtl((ld)(q - 1) / q) * pm1;
    *pq = pqv;
    *pq1 = p;
    *sumsq = s;
}

fk_status gh_rule_impl(int q, double *nodes, double *weights)
{
    if (q < 1 || q > 64) return fail(FK_ERR_ARG, "gh_q must be in [1, 64], got %d", q);
    if (!nodes || !weights) return fail(FK_ERR_ARG, "null output");
    std::vector<ld> x(q), w(q);
    const ld bound = 2.0L * sqrtl((ld)q / 2.0L) + 1.0L;
    for (int i = 0; i < q; ++i) {
        ld lo = -bound, hi = bound;
        for (int it = 0; it < 200 && hi - lo > 0; ++it) {
            ld mid = 0.5L * (lo + hi);
            if (mid == lo || mid == hi) break;
            if (sturm_count(q, mid) > i) hi = mid; else lo = mid;
        }
        ld r = 0.5L * (lo + hi);
        for (int it = 0; it < 3; ++it) {
            ld pq, pq1, s;
            hermite_orthonormal(q, r, &pq, &pq1, &s);
            ld dp = sqrtl(2.0L * q) * pq1;
            if (dp != 0) r -= pq / dp;
        }
        ld pq, pq1, s;
        hermite_orthonormal(q, r, &pq, &pq1, &s);
        x[i] = r;
        w[i] = 1.0L / s;
    }
    const ld sqpi = sqrtl(acosl(-1.0L));
    for (int i = 0; i < q; ++i) {
        ld a = 0.5L * (x[i] - x[q - 1 - i]);
        ld ww = 0.5L * (w[i] + w[q - 1 - i]) / sqpi;
        nodes[i] = (double)a;
        weights[i] = (double)ww;
    }
    if (q % 2 == 1) nodes[q / 2] = 0.0;
    return FK_OK;
}

// ---------------------------------------------------------------------------
// Plan
// ---------------------------------------------------------------------------
struct Region {
    size_t off = 0, bytes = 0;
};

}  // namespace

struct fk_plan {
    std::vector<fk_problem> probs;
    fk_options opt{};
    int n_inst = 0, d = 0, qs = 0, Q = 0, N = 0, n_theta = 0, G = 1;
    double dt = 0, t0 = 0;
    bool f32 = false;
    // host tables
    std::vector<fk::DevInst> inst;
    std::vector<double> coords;
    std::vector<int> active;
    std::vector<unsigned char> cls;
    std::vector<double> gh_a, gh_w, gh_w1;
    std::vector<float> gh_wf, gh_w1f;
    std::vector<double> tfac;
    std::vector<fk::WorkItem> slope_work, node_work, act_work, row_work, split_work;
    std::vector<fk::WorkItem> ell_work;   // non-separable ELL rows by width class
    std::vector<fk::WorkItem> ell_sep_work;   // separable ELL rows, runs of up to 64, by class
    int ell_lmax = 1;                     // longest row box axis
    int n_ell_sep_cls = 0;
    int ell_sep_off[fk::kEllClasses] = {}, ell_sep_n[fk::kEllClasses] = {},
        ell_sep_l[fk::kEllClasses] = {}, ell_sep_tb[fk::kEllClasses] = {};
    int n_ell_cls = 0;
    int ell_cls_off[fk::kEllClasses] = {}, ell_cls_n[fk::kEllClasses] = {},
        ell_cls_w[fk::kEllClasses] = {};
    int tile_elems = 0;
    // adjoint step lists (per-node form and box form by class) with LDS tiles
    struct {
        std::vector<int> fw_nodes, box_nodes;
        std::vector<fk::WorkItem> fw_work, box_work;
        std::vector<fk::TileBox> fw_tiles, box_tiles;
        int box_work_off[fk::kBoxClasses] = {0}, n_box_work[fk::kBoxClasses] = {0};
        int n_in_work = 0;
        // tile staging (see stage_tiles)
        long long stage_entries = 0;
        std::vector<int> cov_node, cov_ptr, cov_base;
    } adj;
    // forward step lists
    std::vector<int> fw_nodes, box_nodes;
    std::vector<fk::WorkItem> fw_work, fw_split_work, box_work;
    int box_work_off[fk::kBoxClasses] = {0}, n_box_work[fk::kBoxClasses] = {0};
    bool use_box = false;
    bool faces = false;   // face kinds other than exit-1, or node-dependent diffusion
    int step_kind = 0;
    int n_table_work = 0;
    std::vector<int64_t> node_off, act_count;
    long long n_nodes = 0, n_active = 0;
    int ell_box[3] = {1, 1, 1};
    int ell_width = 0;
    long long ell_total = 0;     // stored values, with block padding
    long long ell_entries = 0;   // width x active rows, summed over instances
    // measurement: when prof is set, fk_adjoint records a HIP event after
    // every kernel group (kind >= 0) or before one (kind -1)
    std::vector<std::pair<hipEvent_t, int>> *prof = nullptr;
    // workspace
    std::map<std::string, Region> reg;
    size_t ws_bytes = 0;
    size_t ws_fwd_bytes = 0;   // prefix of the workspace that a forward pass uses
    unsigned char *ws = nullptr;
    fk::PlanDev dev{};
    // graph cache
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec = nullptr;
    // checkpoints of u stored by the latest full fk_forward (enqueued on
    // ckpt_stream); fk_adjoint on that stream reuses them
    bool ckpt_valid = false;
    hipStream_t ckpt_stream = nullptr;
    std::string gkey;
    int n_ckpt = 0;
    // instances computed in FP64 inside an FP32 plan (fk_problem.force_f64):
    // they stay in this plan's layout without active nodes, and a child FP64
    // plan over them reads and writes this plan's fields through conversion
    // kernels
    std::vector<unsigned char> skip;   // per instance: handled by the child
    fk_plan *sub = nullptr;            // the child
    std::vector<int> sub_inst;         // child instance k = instance sub_inst[k]
    bool conv = false;                 // this is a child: fields of the parent
    long long out_n_nodes = 0;         // child: nodes of the parent's fields
    std::vector<int> parent_inst;      // child: parent index of each instance

    void *at(const char *name) const { return ws + reg.at(name).off; }
};

namespace {

size_t elt(const fk_plan *p) { return p->f32 ? 4 : 8; }
int rec_stride(int d) { return d == 1 ? 2 : 4; }

bool is_finite(double v) { return std::isfinite(v); }

fk_status validate(const fk_problem &pr, int i)
{
    if (pr.d < 1 || pr.d > 3) return fail(FK_ERR_ARG, "instance %d: d must be 1..3", i);
    for (int a = 0; a < pr.d; ++a) {
        const fk_axis &ax = pr.ax[a];
        if (ax.n < 4) return fail(FK_ERR_ARG, "instance %d axis %d: n must be >= 4", i, a);
        if (!ax.nodes) return fail(FK_ERR_ARG, "instance %d axis %d: null nodes", i, a);
        for (int k = 0; k < ax.n; ++k)
            if (!is_finite(ax.nodes[k]))
                return fail(FK_ERR_NONFINITE, "instance %d axis %d: non-finite node", i, a);
        for (int k = 1; k < ax.n; ++k)
            if (!(ax.nodes[k] > ax.nodes[k - 1]))
                return fail(FK_ERR_ARG, "instance %d axis %d: nodes not strictly increasing", i, a);
    }
    long long J = 1;
    for (int a = 0; a < pr.d; ++a) J *= pr.ax[a].n;
    if (J > (1LL << 29)) return fail(FK_ERR_UNSUPPORTED, "instance %d: more than 2^29 nodes", i);
    if (pr.coef_kind < 0 || pr.coef_kind > 4) return fail(FK_ERR_ARG, "instance %d: coef_kind", i);
    if (pr.coef_kind == FK_COEF_RUNAWAY3D && pr.d != 3)
        return fail(FK_ERR_ARG, "instance %d: the runaway model needs d = 3", i);
    if (pr.coef_kind == FK_COEF_RUNAWAY3D &&
        !(pr.ax[0].nodes[0] > 0 && pr.ax[1].nodes[0] >= -1 && pr.ax[1].nodes[pr.ax[1].n - 1] <= 1))
        return fail(FK_ERR_ARG, "instance %d: the runaway model needs p > 0 and xi in [-1, 1]", i);
    for (int a = 0; a < pr.d; ++a)
        for (int sd = 0; sd < 2; ++sd) {
            const int f = pr.face[a][sd];
            if (f < FK_FACE_EXIT1 || f > FK_FACE_REFLECT)
                return fail(FK_ERR_ARG, "instance %d axis %d: face kind %d", i, a, f);
            if (f != FK_FACE_EXIT1 && pr.ax[a].periodic)
                return fail(FK_ERR_ARG, "instance %d axis %d: a periodic axis has no faces", i, a);
        }
    if (pr.coef_kind == FK_COEF_ROLLS2D && pr.d != 2)
        return fail(FK_ERR_ARG, "instance %d: roll flow needs d = 2", i);
    if (pr.coef_kind == FK_COEF_CELLULAR2D && pr.d != 2)
        return fail(FK_ERR_ARG, "instance %d: cellular flow needs d = 2", i);
    if (pr.coef_kind == FK_COEF_ABC3D && pr.d != 3)
        return fail(FK_ERR_ARG, "instance %d: ABC flow needs d = 3", i);
    for (int k = 0; k < 16; ++k)
        if (!is_finite(pr.coef[k])) return fail(FK_ERR_NONFINITE, "instance %d: non-finite coef", i);
    if (!is_finite(pr.D) || !is_finite(pr.dt) || !is_finite(pr.t0))
        return fail(FK_ERR_NONFINITE, "instance %d: non-finite D, dt or t0", i);
    if (pr.D < 0) return fail(FK_ERR_ARG, "instance %d: D must be >= 0", i);
    if (!(pr.dt > 0)) return fail(FK_ERR_ARG, "instance %d: dt must be > 0", i);
    if (pr.n_steps < 1) return fail(FK_ERR_ARG, "instance %d: n_steps must be >= 1", i);
    if (pr.gh_q < 1 || pr.gh_q > 64) return fail(FK_ERR_ARG, "instance %d: gh_q in [1, 64]", i);
    if (pr.region_kind != FK_REGION_BOX && pr.region_kind != FK_REGION_BALL)
        return fail(FK_ERR_ARG, "instance %d: region_kind", i);
    if (pr.region_kind == FK_REGION_BALL) {
        if (!(pr.radius > 0) || !is_finite(pr.radius))
            return fail(FK_ERR_ARG, "instance %d: ball radius must be > 0", i);
        for (int a = 0; a < pr.d; ++a) {
            if (pr.ax[a].periodic) return fail(FK_ERR_UNSUPPORTED, "instance %d: ball with periodic axis", i);
            const double lo = pr.ax[a].nodes[0], hi = pr.ax[a].nodes[pr.ax[a].n - 1];
            if (!(pr.center[a] - pr.radius >= lo && pr.center[a] + pr.radius <= hi))
                return fail(FK_ERR_ARG, "instance %d: ball not inside the grid box", i);
        }
    }
    return FK_OK;
}

bool axis_uniform(const fk_axis &ax)
{
    const double lo = ax.nodes[0], hi = ax.nodes[ax.n - 1];
    const double h = (hi - lo) / (ax.n - 1);
    for (int k = 0; k < ax.n; ++k)
        if (std::fabs(ax.nodes[k] - (lo + k * h)) > 1e-9 * h) return false;
    return true;
}

// x_k == k * step + lo exactly for k < n-1 and x_{n-1} == hi, with the same
// operations as the kernels' coordinate formula (no contraction).
bool axis_affine(const fk_axis &ax, double *step_out)
{
    const double lo = ax.nodes[0], hi = ax.nodes[ax.n - 1];
    const double step = (hi - lo) / (double)(ax.n - 1);
    *step_out = step;
    for (int k = 0; k < ax.n - 1; ++k) {
        const double xk = (double)k * step + lo;
        if (xk != ax.nodes[k]) return false;
    }
    return true;
}

// Largest |b_a| the drift can take (bounds the reach of landing points).
double drift_bound(const fk_problem &pr, int a)
{
    const double *c = pr.coef;
    if (pr.coef_kind == FK_COEF_CONST) return std::fabs(c[a]);
    if (pr.coef_kind == FK_COEF_CELLULAR2D) return std::fabs(c[0]) * M_PI;
    if (pr.coef_kind == FK_COEF_ROLLS2D)
        return std::fabs(c[0]) * (a == 0 ? M_PI : std::fabs(c[3])) * (1.0 + std::fabs(c[1]));
    const double f = 1.0 + std::fabs(c[3]);
    if (a == 0) return (std::fabs(c[0]) + std::fabs(c[2])) * f;
    if (a == 1) return (std::fabs(c[1]) + std::fabs(c[0])) * f;
    return (std::fabs(c[2]) + std::fabs(c[1])) * f;
}

// Exit value of a point (-1: none), the same comparisons as the kernels:
// faces by the lowest axis, low face first, then the ball (value 1).
int exit_value(const fk_problem &pr, const double *z)
{
    for (int a = 0; a < pr.d; ++a) {
        if (pr.ax[a].periodic) continue;
        const int fl = pr.face[a][0], fh = pr.face[a][1];
        if (fl != FK_FACE_REFLECT && z[a] <= pr.ax[a].nodes[0]) return fl == FK_FACE_EXIT0 ? 0 : 1;
        if (fh != FK_FACE_REFLECT && z[a] >= pr.ax[a].nodes[pr.ax[a].n - 1])
            return fh == FK_FACE_EXIT0 ? 0 : 1;
    }
    if (pr.region_kind == FK_REGION_BALL) {
        double s = 0.0;
        for (int a = 0; a < pr.d; ++a) {
            const double t = z[a] - pr.center[a];
            const double t2 = t * t;
            s = s + t2;
        }
        if (s >= pr.radius * pr.radius) return 1;
    }
    return -1;
}

// Runaway-electron model (Section 4.3): the time factors (E, nu_ee, v_T,
// delta) at t -- constants, or the thermal-quench model when t_* > 0 --
// and, at node x, the drift and the per-axis diffusion coefficients (the
// formulas of the kernels' runaway_centre; used for the reach bound).
void runaway_time_factors(const fk_problem &pr, double t, double *tf)
{
    const double *p = pr.coef;
    if (p[11] > 0.0) {
        const double Th = p[13] + (p[12] - p[13]) * std::exp(-t / p[11]);
        const double lnh = 14.9 - 0.5 * std::log(0.28) + std::log(Th);
        const double lnt = 14.9 - 0.5 * std::log(0.28) + std::log(p[14]);
        tf[2] = std::sqrt(Th / p[14]);
        tf[1] = std::pow(p[14] / Th, 1.5) * lnh / lnt;
        tf[3] = std::sqrt(2.0 * Th / p[15]);
        tf[0] = p[0] * std::pow(p[12] / Th, 1.5);
    } else {
        tf[0] = p[0]; tf[1] = p[4]; tf[2] = p[5]; tf[3] = p[3];
    }
}

void runaway_coefficients(const fk_problem &pr, const double *tf, const double *x, double *b,
                          double *sig)
{
    const double *p = pr.coef;
    const double E = tf[0], nu = tf[1], vT = tf[2], delta = tf[3];
    const double pm = x[0], xi = x[1], r = x[2];
    const double gam = std::sqrt(1.0 + (delta * pm) * (delta * pm));
    const double om = 1.0 - xi * xi;
    const double y = pm / gam;
    const double phi = std::erf(y);
    const double dphi = 2.0 / std::sqrt(M_PI) * std::exp(-y * y);
    const double psi = (phi - y * dphi) / (2.0 * y * y);
    const double dpsi = dphi - 2.0 * psi / y;
    const double k2 = nu * vT * vT;
    const double CA = k2 * psi / y;
    const double CB = 0.5 * k2 / y * (p[2] + phi - psi + 0.5 * y * y * std::pow(delta, 4.0));
    const double CF = 2.0 * nu * vT * psi;
    const double dCA = k2 * (dpsi * y - psi) / (y * y) / (gam * gam * gam);
    const double th = std::tanh((r - p[6]) / p[7]);
    const double ep = std::exp(-(pm / p[8]) * (pm / p[8]));
    const double Dr = 0.5 * p[10] * (1.0 + th) * ep;
    const double dDr = 0.5 * p[10] * (1.0 - th * th) / p[7] * ep;
    b[0] = E * xi - gam * pm / p[1] * om - CF + 2.0 * CA / pm + dCA;
    b[1] = E * om / pm - xi * om / (p[1] * gam) - 2.0 * xi * CB / (pm * pm);
    b[2] = (r > p[6] ? p[9] : 0.0) + dDr;
    sig[0] = std::sqrt(2.0 * CA);
    sig[1] = std::sqrt(2.0 * CB) / pm * std::sqrt(om > 0.0 ? om : 0.0);
    sig[2] = std::sqrt(2.0 * Dr);
}

// Largest |b_a| and sigma_a of the runaway model over the instance's nodes,
// at the first and the last step, doubled (bounds the reach of its landing
// points; the active region of this model is the whole grid anyway).
void runaway_bounds(const fk_problem &pr, double *bmax, double *smax)
{
    for (int a = 0; a < 3; ++a) bmax[a] = smax[a] = 0.0;
    for (int e = 0; e < 2; ++e) {
        double tf[4];
        runaway_time_factors(pr, pr.t0 + (e ? pr.n_steps - 1 : 0) * pr.dt, tf);
        double x[3], b[3], sg[3];
        for (int i = 0; i < pr.ax[0].n; ++i)
            for (int j = 0; j < pr.ax[1].n; ++j)
                for (int k = 0; k < pr.ax[2].n; ++k) {
                    x[0] = pr.ax[0].nodes[i]; x[1] = pr.ax[1].nodes[j]; x[2] = pr.ax[2].nodes[k];
                    runaway_coefficients(pr, tf, x, b, sg);
                    for (int a = 0; a < 3; ++a) {
                        bmax[a] = std::max(bmax[a], std::fabs(b[a]));
                        smax[a] = std::max(smax[a], sg[a]);
                    }
                }
    }
    for (int a = 0; a < 3; ++a) { bmax[a] *= 2.0; smax[a] *= 2.0; }
}

void add_region(fk_plan *p, const char *name, size_t bytes)
{
    Region r;
    r.off = p->ws_bytes;
    r.bytes = bytes;
    p->reg[name] = r;
    p->ws_bytes = align_up(p->ws_bytes + std::max<size_t>(bytes, 1));
}

// Staging of the adjoint's LDS tiles.  Tiles of neighbouring work items
// overlap (each is its node box widened by the reach), so adding them to mu
// directly takes device-wide atomics.  Instead every tile that fits LDS gets
// a slot of its own (entries in row-major tile order, the d + 1 fields of an
// entry adjacent), written with plain stores, and each node gets the list of
// slot entries that hold it; k_gather_tiles sums those lists into mu.  Plans
// whose slots would pass 2^31 entries keep the atomic flush.
void stage_tiles(fk_plan *p)
{
    const int d = p->d, NF = d + 1;
    auto &A = p->adj;
    A.stage_entries = 0;
    A.cov_node.clear();
    A.cov_ptr.clear();
    A.cov_base.clear();
    long long off = 0;
    auto assign = [&](std::vector<fk::TileBox> &tiles) {
        for (fk::TileBox &tb : tiles) {
            tb.soff = -1;
            if (!tb.use_lds) continue;
            long long cells = 1;
            for (int a = 0; a < d; ++a) cells *= tb.ext[a];
            tb.soff = (int)std::min<long long>(off, INT_MAX);
            off += cells * NF;
        }
    };
    assign(A.fw_tiles);
    assign(A.box_tiles);
    if (off == 0 || off > (long long)INT_MAX || p->n_nodes > (long long)INT_MAX) {
        for (fk::TileBox &tb : A.fw_tiles) tb.soff = -1;
        for (fk::TileBox &tb : A.box_tiles) tb.soff = -1;
        return;
    }
    A.stage_entries = off;
    // each tile entry's packed node (periodic tiles may run past the seam)
    auto visit = [&](const std::vector<fk::TileBox> &tiles, const std::vector<fk::WorkItem> &work,
                     auto &&fn) {
        for (size_t t = 0; t < tiles.size(); ++t) {
            const fk::TileBox &tb = tiles[t];
            if (tb.soff < 0) continue;
            const fk_problem &pr = p->probs[work[t].inst];
            long long stride[3] = {1, 1, 1};
            for (int a = d - 2; a >= 0; --a) stride[a] = stride[a + 1] * pr.ax[a + 1].n;
            const int e0 = tb.ext[0], e1 = d > 1 ? tb.ext[1] : 1, e2 = d > 2 ? tb.ext[2] : 1;
            int c = 0;
            for (int l0 = 0; l0 < e0; ++l0)
                for (int l1 = 0; l1 < e1; ++l1)
                    for (int l2 = 0; l2 < e2; ++l2, ++c) {
                        const int l[3] = {l0, l1, l2};
                        long long node = p->node_off[work[t].inst];
                        for (int a = 0; a < d; ++a) {
                            const int n = pr.ax[a].n;
                            int i = tb.lo[a] + l[a];
                            if (pr.ax[a].periodic) {
                                if (i < 0) i += n - 1;
                                else if (i > n - 1) i -= n - 1;
                            }
                            node += (long long)i * stride[a];
                        }
                        fn(node, tb.soff + c * NF);
                    }
        }
    };
    // counting sort by node, then the covered nodes only
    std::vector<int> cnt((size_t)p->n_nodes + 1, 0);
    auto count = [&](long long node, int) { ++cnt[(size_t)node + 1]; };
    visit(A.fw_tiles, A.fw_work, count);
    visit(A.box_tiles, A.box_work, count);
    for (size_t j = 0; j < (size_t)p->n_nodes; ++j) cnt[j + 1] += cnt[j];
    A.cov_base.assign((size_t)cnt[(size_t)p->n_nodes], 0);
    std::vector<int> fill(cnt.begin(), cnt.end() - 1);
    auto put = [&](long long node, int base) { A.cov_base[(size_t)fill[(size_t)node]++] = base; };
    visit(A.fw_tiles, A.fw_work, put);
    visit(A.box_tiles, A.box_work, put);
    for (size_t j = 0; j < (size_t)p->n_nodes; ++j)
        if (cnt[j + 1] > cnt[j]) {
            A.cov_node.push_back((int)j);
            A.cov_ptr.push_back(cnt[j]);
        }
    A.cov_ptr.push_back(cnt[(size_t)p->n_nodes]);
}

void build_work(std::vector<fk::WorkItem> &out, int inst, int count, int chunk, int first = 0,
                int kind = 0)
{
    for (int f = 0; f < count; f += chunk) {
        fk::WorkItem w;
        w.inst = inst;
        w.first = first + f;
        w.count = std::min(chunk, count - f);
        w.kind = kind;
        out.push_back(w);
    }
}

int grid_for(size_t n_work, int per_cu = 8)
{
    // persistent grid: enough workgroups for the work list, at most per_cu per
    // CU (8 for 256-thread workgroups), a multiple of the 8 XCDs
    size_t g = std::min<size_t>(n_work, (size_t)256 * per_cu);
    if (g >= 8) g = (g + 7) / 8 * 8;
    return (int)std::max<size_t>(g, 1);
}

fk_status build_plan(fk_plan *p)
{
    const fk_problem &p0 = p->probs[0];
    p->d = p0.d;
    p->qs = p0.gh_q;
    p->N = p0.n_steps;
    p->dt = p0.dt;
    p->t0 = p0.t0;
    p->Q = 1;
    for (int a = 0; a < p->d; ++a) p->Q *= p->qs;
    // lanes per active node: the tensor points spread over at most one wave, and
    // at least d Q* lanes for the per-axis staging of the step pass
    p->G = std::max(4, std::min(64, group_of(p->Q)));
    if (p->d * p->qs > p->G) return fail(FK_ERR_UNSUPPORTED, "d * gh_q above the lane group");
    p->n_theta = (p0.coef_kind == FK_COEF_CONST) ? p->d + 1
               : (p0.coef_kind == FK_COEF_ABC3D ? 5
               : (p0.coef_kind == FK_COEF_RUNAWAY3D ? 1 : 4));
    for (const fk_problem &pr : p->probs) {
        p->faces = p->faces || pr.coef_kind == FK_COEF_RUNAWAY3D;
        for (int a = 0; a < pr.d; ++a)
            p->faces = p->faces || pr.face[a][0] != FK_FACE_EXIT1 || pr.face[a][1] != FK_FACE_EXIT1;
    }
    if ((long long)p->Q > 256) return fail(FK_ERR_UNSUPPORTED, "Q = gh_q^d above 256");

    p->gh_a.assign(p->qs, 0.0);
    std::vector<double> w1(p->qs);
    fk_status st = gh_rule_impl(p->qs, p->gh_a.data(), w1.data());
    if (st != FK_OK) return st;
    p->gh_w1 = w1;
    p->gh_w1f.assign(w1.begin(), w1.end());
    p->gh_w.assign(p->Q, 0.0);
    p->gh_wf.assign(p->Q, 0.0f);
    for (int q = 0; q < p->Q; ++q) {
        int qi[3], r = q;
        for (int a = p->d - 1; a >= 0; --a) { qi[a] = r % p->qs; r /= p->qs; }
        double w = w1[qi[0]];
        for (int a = 1; a < p->d; ++a) w = w * w1[qi[a]];
        p->gh_w[q] = w;
        p->gh_wf[q] = (float)w;
    }
    double amax = 0.0;
    for (double a : p->gh_a) amax = std::max(amax, std::fabs(a));

    const int npb = kBlock / p->G;
    std::vector<fk::WorkItem> tables, runs;
    long long ell_total = 0, ell_wmax = 0, ell_rows_w = 0;
    std::vector<std::vector<int>> inst_sep, inst_rest;
    std::vector<int> inst_cls, inst_lneed;
    std::vector<std::vector<unsigned char>> inst_inner;   // per node: no landing point can exit
    std::vector<std::vector<unsigned char>> inst_seprow;  // per active row: separable
    std::vector<std::array<int, 3>> inst_dils;
    p->node_off.assign(p->n_inst + 1, 0);
    p->act_count.assign(p->n_inst, 0);
    long long coord_total = 0;
    int box[3] = {1, 1, 1};
    for (int i = 0; i < p->n_inst; ++i) {
        const fk_problem &pr = p->probs[i];
        fk::DevInst I;
        std::memset(&I, 0, sizeof(I));
        I.d = pr.d;
        long long J = 1;
        for (int a = 0; a < pr.d; ++a) J *= pr.ax[a].n;
        long long stride = 1;
        for (int a = pr.d - 1; a >= 0; --a) {
            I.stride[a] = stride;
            stride *= pr.ax[a].n;
        }
        for (int a = 0; a < 3; ++a) {
            if (a < pr.d) {
                const fk_axis &ax = pr.ax[a];
                I.n[a] = ax.n;
                I.periodic[a] = ax.periodic ? 1 : 0;
                I.uniform[a] = axis_uniform(ax) ? 1 : 0;
                double step = 0.0;
                I.affine[a] = axis_affine(ax, &step) ? 1 : 0;
                I.step[a] = step;
                I.coord_off[a] = coord_total;
                I.lo[a] = ax.nodes[0];
                I.hi[a] = ax.nodes[ax.n - 1];
                I.period[a] = ax.nodes[ax.n - 1] - ax.nodes[0];
                I.inv_h[a] = I.affine[a] ? 1.0 / step
                                         : (ax.n - 1) / (ax.nodes[ax.n - 1] - ax.nodes[0]);
                for (int k = 0; k < ax.n; ++k) p->coords.push_back(ax.nodes[k]);
                coord_total += ax.n;
            } else {
                I.n[a] = 1;
            }
        }
        I.coef_kind = pr.coef_kind;
        I.region_kind = pr.region_kind;
        for (int k = 0; k < 16; ++k) I.coef[k] = pr.coef[k];
        I.D = pr.D;
        for (int a = 0; a < 3; ++a) I.center[a] = pr.center[a];
        I.r2 = pr.radius * pr.radius;
        const double sq = std::sqrt(2.0 * pr.dt);
        I.S = std::sqrt(2.0 * pr.D) * sq;
        I.dSdD = pr.D > 0 ? I.S / (2.0 * pr.D) : 0.0;
        double re_bmax[3] = {0, 0, 0}, re_smax[3] = {0, 0, 0};
        if (pr.coef_kind == FK_COEF_RUNAWAY3D) {
            runaway_bounds(pr, re_bmax, re_smax);
            I.sdiff = 1;
            I.S = 0.0;
            I.dSdD = 0.0;
        }
        for (int a = 0; a < 3; ++a)
            for (int sd = 0; sd < 2; ++sd) I.face[a][sd] = a < pr.d ? pr.face[a][sd] : 0;
        I.node_off = p->n_nodes;
        I.out_off = p->n_nodes;
        I.act_off = p->n_active;
        const bool skip_i = !p->skip.empty() && p->skip[i];

        // node classes: 0 active, 1 exit, 2 image of active, 3 image of exit
        std::vector<unsigned char> c(J);
        int idx[3];
        double x[3];
        for (long long j = 0; j < J; ++j) {
            long long r = j;
            for (int a = pr.d - 1; a >= 0; --a) { idx[a] = (int)(r % pr.ax[a].n); r /= pr.ax[a].n; }
            bool image = false;
            for (int a = 0; a < pr.d; ++a)
                if (pr.ax[a].periodic && idx[a] == pr.ax[a].n - 1) { image = true; idx[a] = 0; }
            for (int a = 0; a < pr.d; ++a) x[a] = pr.ax[a].nodes[idx[a]];
            const int ev = skip_i ? 1 : exit_value(pr, x);
            c[j] = (unsigned char)((image ? 2 : 0) | (ev >= 0 ? 1 : 0) | (ev == 0 ? 4 : 0));
        }
        int na = 0;
        int amin[3] = {1 << 30, 1 << 30, 1 << 30}, amax_i[3] = {-1, -1, -1};
        for (long long j = 0; j < J; ++j)
            if (c[j] == 0) {
                p->active.push_back((int)j);
                na++;
                long long r = j;
                for (int a = pr.d - 1; a >= 0; --a) {
                    const int ia = (int)(r % pr.ax[a].n);
                    r /= pr.ax[a].n;
                    amin[a] = std::min(amin[a], ia);
                    amax_i[a] = std::max(amax_i[a], ia);
                }
            }
        // trig tables of the drift arguments, one entry per axis coordinate
        if (pr.coef_kind != FK_COEF_CONST && pr.coef_kind != FK_COEF_RUNAWAY3D)
            for (int a = 0; a < pr.d; ++a)
                build_work(tables, i, pr.ax[a].n, kBlock, 0, 1 + a);
        // slope records are needed only where landing cells of active nodes can
        // reach: the active bounding box widened by the reach plus the corner
        int blo[3] = {0, 0, 0}, bhi[3] = {0, 0, 0};
        int dils[3] = {0, 0, 0};
        for (int a = 0; a < pr.d; ++a) {
            double hmin = 1e300;
            for (int k = 1; k < pr.ax[a].n; ++k)
                hmin = std::min(hmin, pr.ax[a].nodes[k] - pr.ax[a].nodes[k - 1]);
            const double reach = pr.coef_kind == FK_COEF_RUNAWAY3D
                ? re_bmax[a] * pr.dt + re_smax[a] * std::sqrt(2.0 * pr.dt) * amax
                : drift_bound(pr, a) * pr.dt + I.S * amax;
            const double cells = std::ceil(reach / hmin) + 2.0;
            const int dil = cells > 1e9 ? (1 << 30) : (int)cells;
            // a landing cell lies within ceil(reach / h) cells of its node, and
            // its upper corner one further: the adjoint tile's halo
            dils[a] = std::min(dil - 1, pr.ax[a].n);
            if (pr.ax[a].periodic || na == 0) {
                blo[a] = 0;
                bhi[a] = pr.ax[a].n - 1;
            } else {
                blo[a] = std::max(0, amin[a] - dil);
                bhi[a] = (int)std::min<long long>(pr.ax[a].n - 1, (long long)amax_i[a] + dil);
            }
        }
        if (na > 0) {
            const int dl = pr.d - 1;
            long long rows = 1;
            for (int a = 0; a < dl; ++a) rows *= (bhi[a] - blo[a] + 1);
            for (long long r = 0; r < rows; ++r) {
                long long rr = r, base = 0;
                for (int a = dl - 1; a >= 0; --a) {
                    const int len = bhi[a] - blo[a] + 1;
                    const int ia = blo[a] + (int)(rr % len);
                    rr /= len;
                    base += (long long)ia * I.stride[a];
                }
                build_work(runs, i, bhi[dl] - blo[dl] + 1, kBlock, (int)(base + blo[dl]), 0);
            }
        }
        p->cls.insert(p->cls.end(), c.begin(), c.end());
        I.n_act = na;
        p->inst.push_back(I);
        p->node_off[i] = p->n_nodes;
        p->act_count[i] = na;
        build_work(p->node_work, i, (int)J, kBlock);
        build_work(p->act_work, i, na, npb);
        // separable nodes: every active node of a box region; for a ball, nodes
        // whose landing points stay strictly inside it (distance + reach < r)
        {
            double reach2 = 0.0;
            for (int a = 0; a < pr.d; ++a) {
                const double ra = drift_bound(pr, a) * pr.dt + I.S * amax;
                reach2 += ra * ra;
            }
            const double reach = std::sqrt(reach2);
            int Lneed = 0;
            for (int a = 0; a < pr.d; ++a) {
                double hmin = 1e300;
                for (int k = 1; k < pr.ax[a].n; ++k)
                    hmin = std::min(hmin, pr.ax[a].nodes[k] - pr.ax[a].nodes[k - 1]);
                Lneed = std::max(Lneed, (int)std::floor(2.0 * I.S * amax / hmin) + 3);
            }
            static const int kL[fk::kBoxClasses] = {3, 4, 5, 6, 8};
            int cls_box = -1;
            for (int c2 = 0; c2 < fk::kBoxClasses; ++c2)
                if (Lneed <= kL[c2]) { cls_box = c2; break; }
            std::vector<int> sep, rest;
            std::vector<unsigned char> inner(J, 0);
            std::vector<unsigned char> seprow(na, 0);
            double reach_a[3] = {0, 0, 0};
            for (int a = 0; a < pr.d; ++a) reach_a[a] = drift_bound(pr, a) * pr.dt + I.S * amax;
            for (int t = 0; t < na; ++t) {
                const int j = p->active[I.act_off + t];
                bool separable = true;
                // interior: no landing point can leave the box on a non-periodic
                // axis (with a relative margin for the rounding of z), nor the ball
                bool interior = true;
                long long r = j;
                double dist2 = 0.0;
                for (int a = pr.d - 1; a >= 0; --a) {
                    const int ia = (int)(r % pr.ax[a].n);
                    r /= pr.ax[a].n;
                    const double x = pr.ax[a].nodes[ia];
                    const double dx = x - pr.center[a];
                    dist2 += dx * dx;
                    if (!pr.ax[a].periodic) {
                        const double lo = pr.ax[a].nodes[0], hi = pr.ax[a].nodes[pr.ax[a].n - 1];
                        const double m = reach_a[a] * (1.0 + 1e-6) + 1e-12 * (hi - lo);
                        interior = interior && x - m > lo && x + m < hi;
                    }
                }
                if (pr.region_kind == FK_REGION_BALL) {
                    separable = std::sqrt(dist2) + reach < pr.radius * (1.0 - 1e-9);
                    interior = interior && separable;
                }
                inner[j] = interior ? 1 : 0;
                seprow[t] = separable ? 1 : 0;
                (separable ? sep : rest).push_back(j);
            }
            inst_inner.push_back(std::move(inner));
            inst_seprow.push_back(std::move(seprow));
            inst_sep.push_back(sep);
            inst_rest.push_back(rest);
            inst_cls.push_back(cls_box);
            inst_lneed.push_back(Lneed);
        }
        build_work(p->row_work, i, na, kBlock);
        inst_dils.push_back({dils[0], dils[1], dils[2]});
        build_work(p->split_work, i, na, kBlock / std::max(2, group_of(p->qs)));
        p->n_nodes += J;
        p->n_active += na;

        // ELL row box: the landing points of one node spread over 2 S max|a|
        {
            long long Wi = pr.d + 1;
            for (int a = 0; a < pr.d; ++a) {
                double hmin = 1e300;
                for (int k = 1; k < pr.ax[a].n; ++k)
                    hmin = std::min(hmin, pr.ax[a].nodes[k] - pr.ax[a].nodes[k - 1]);
                int L = (int)std::floor(2.0 * I.S * amax / hmin) + 3;
                L = std::min(L, pr.ax[a].n);
                p->inst.back().ell_box[a] = L;
                box[a] = std::max(box[a], L);
                Wi *= L;
            }
            for (int a = pr.d; a < 3; ++a) p->inst.back().ell_box[a] = 1;
            // values are stored in 16-byte blocks of consecutive box nodes of
            // one field (4 in FP32, 2 in FP64); the box is padded to whole blocks
            const long long KB = p->opt.precision == FK_PREC_F32 ? 4 : 2;
            const long long nbox = Wi / (pr.d + 1);
            const long long nbp = (nbox + KB - 1) / KB * KB;
            p->inst.back().ell_w = (int)Wi;
            p->inst.back().ell_nbp = (int)nbp;
            p->inst.back().ell_off = ell_total;
            ell_total += (pr.d + 1) * nbp * na;
            ell_rows_w += Wi * na;
            ell_wmax = std::max(ell_wmax, Wi);
        }
    }
    p->node_off[p->n_inst] = p->n_nodes;
    // forward step layout: thread per node for large plans (with the box form
    // for separable nodes), Q* lanes per node for small ones
    {
        const int sk = p->opt.step_kernel;
        const bool large = p->n_active >= 256LL * 4 * 64 * 2;
        const bool node_ok = fk::step_node_compiled(p->d, p->qs);
        bool affine = true;
        for (const fk::DevInst &I : p->inst)
            for (int a = 0; a < p->d; ++a) affine = affine && I.affine[a];
        // faces (other than exit-1) with the R2 interpolant: the lane-group step
        const bool faces_r2 = p->faces && p->opt.hermite == FK_HERMITE_R2;
        if (sk == 2 || !node_ok || faces_r2) p->step_kind = 1;
        else if (sk == 3 || (sk == 0 && !large)) p->step_kind = 2;
        else p->step_kind = 0;
        // the separable form by default in 3D only: there a node's Q*^3
        // points gather 8 corners each, against L^3 records of its footprint;
        // in 2D (Q*^2 points x 4 corners vs L^2) the per-point gather is faster
        // the R2 interpolant in 3D: thread-per-node kernels only (the 2D box
        // and lane-group forms carry the 2D twist)
        const bool r2 = p->opt.hermite == FK_HERMITE_R2 && p->d == 3;
        p->use_box = node_ok && affine && !p->faces && !r2 && fk::box_compiled(p->d, p->qs) &&
                     (sk == 4 || (sk == 0 && large && p->d == 3));
        const int gs = std::max(2, group_of(p->qs));
        std::vector<std::vector<fk::WorkItem>> bw(fk::kBoxClasses);
        // node lists in patch order (16x16 in 2D, 4x8x8 in 3D, 256 in 1D):
        // a work item never straddles a patch, so its landing footprint (and
        // the adjoint's LDS tile of mu) stays compact
        static const int kPatch[3][3] = {{256, 1, 1}, {16, 16, 1}, {4, 8, 8}};
        auto patch_sort = [&](std::vector<int> &list, const fk_problem &pr,
                              std::vector<long long> &keys) {
            const int *pd = kPatch[pr.d - 1];
            std::vector<std::pair<long long, int>> kv;
            kv.reserve(list.size());
            for (int j : list) {
                long long r = j, key = 0;
                int ia[3];
                for (int a = pr.d - 1; a >= 0; --a) {
                    ia[a] = (int)(r % pr.ax[a].n);
                    r /= pr.ax[a].n;
                }
                for (int a = 0; a < pr.d; ++a) {
                    const int np = (pr.ax[a].n + pd[a] - 1) / pd[a];
                    key = key * np + ia[a] / pd[a];
                }
                kv.push_back({key * (1LL << 31) + j, j});
            }
            std::sort(kv.begin(), kv.end());
            keys.clear();
            for (size_t t = 0; t < kv.size(); ++t) {
                list[t] = kv[t].second;
                keys.push_back(kv[t].first >> 31);
            }
        };
        auto patch_work = [&](std::vector<fk::WorkItem> &out, int inst, const std::vector<long long> &keys,
                              int first, int chunk) {
            size_t t = 0;
            while (t < keys.size()) {
                size_t e = t;
                while (e < keys.size() && keys[e] == keys[t] && (int)(e - t) < chunk) ++e;
                fk::WorkItem w;
                w.inst = inst;
                w.first = first + (int)t;
                w.count = (int)(e - t);
                w.kind = 0;
                out.push_back(w);
                t = e;
            }
        };
        std::vector<long long> keys;
        for (int i = 0; i < p->n_inst; ++i) {
            const fk_problem &pr = p->probs[i];
            std::vector<int> fw = inst_rest[i];
            // the box form up to 5-node footprints: from L = 6 on the box step's
            // vectors no longer fit the registers (measured on 65^3 ABC flows:
            // L = 3 and 5 six and four times faster than a thread per node, L = 6
            // five times slower)
            if (!p->use_box || inst_cls[i] < 0 || inst_cls[i] > 2) {
                fw.insert(fw.end(), inst_sep[i].begin(), inst_sep[i].end());
            } else {
                std::vector<int> sep = inst_sep[i];
                patch_sort(sep, pr, keys);
                const int f0 = (int)p->box_nodes.size();
                p->box_nodes.insert(p->box_nodes.end(), sep.begin(), sep.end());
                patch_work(bw[inst_cls[i]], i, keys, f0, kBlock);
            }
            patch_sort(fw, pr, keys);
            const int f1 = (int)p->fw_nodes.size();
            p->fw_nodes.insert(p->fw_nodes.end(), fw.begin(), fw.end());
            const size_t w0 = p->fw_work.size(), ws0 = p->fw_split_work.size();
            patch_work(p->fw_work, i, keys, f1, kBlock);
            patch_work(p->fw_split_work, i, keys, f1, kBlock / gs);
            // kind 1: no landing point of any node of the item can exit
            auto mark = [&](std::vector<fk::WorkItem> &v, size_t from) {
                for (size_t t = from; t < v.size(); ++t) {
                    bool all = true;
                    for (int u = 0; u < v[t].count && all; ++u)
                        all = inst_inner[i][p->fw_nodes[v[t].first + u]] != 0;
                    v[t].kind = all ? 1 : 0;
                }
            };
            mark(p->fw_work, w0);
            mark(p->fw_split_work, ws0);
        }
        for (int c2 = 0; c2 < fk::kBoxClasses; ++c2) {
            p->box_work_off[c2] = (int)p->box_work.size();
            p->n_box_work[c2] = (int)bw[c2].size();
            p->box_work.insert(p->box_work.end(), bw[c2].begin(), bw[c2].end());
        }
        // adjoint LDS tiles: node box of each work item widened by the reach,
        // d + 1 field planes, innermost axis padded to a pitch that puts the
        // rows of a wave's patch (16 nodes in 2D, 8 in 3D) on distinct banks
        const int NF = p->d + 1;
        const size_t elt_b = 8;   // tiles accumulate in FP64 in both precisions
        const size_t budget = 60 * 1024;   // plus static LDS, within 64 KB per workgroup
        // wrap: a periodic axis' tile may run past the seam (unwrapped indices,
        // less than one period long); the kernel then indexes it unwrapped
        auto tile_of = [&](const fk::WorkItem &it, const std::vector<int> &list, bool wrap) {
            const fk_problem &pr = p->probs[it.inst];
            int mn[3] = {1 << 30, 1 << 30, 1 << 30}, mx[3] = {-1, -1, -1};
            for (int t = 0; t < it.count; ++t) {
                long long r = list[it.first + t];
                for (int a = pr.d - 1; a >= 0; --a) {
                    const int ia = (int)(r % pr.ax[a].n);
                    r /= pr.ax[a].n;
                    mn[a] = std::min(mn[a], ia);
                    mx[a] = std::max(mx[a], ia);
                }
            }
            fk::TileBox tb;
            std::memset(&tb, 0, sizeof(tb));
            bool ok = it.count > 0;
            size_t elems = NF;
            for (int a = 0; a < pr.d; ++a) {
                const int dil = inst_dils[it.inst][a];
                int lo = mn[a] - dil, hi = mx[a] + dil;
                if (pr.ax[a].periodic && (lo < 0 || hi > pr.ax[a].n - 1)) {
                    if (!wrap || hi - lo + 1 > pr.ax[a].n - 1) ok = false;
                } else {
                    lo = std::max(lo, 0);
                    hi = std::min(hi, pr.ax[a].n - 1);
                }
                tb.lo[a] = lo;
                tb.ext[a] = std::max(hi - lo + 1, 1);
                if (a < pr.d - 1) elems *= (size_t)tb.ext[a];
            }
            for (int a = pr.d; a < 3; ++a) tb.ext[a] = 1;
            // pitch of the innermost axis: in 2D and 3D, the next length that is
            // 16 (2D) or 8 (3D) modulo 32 words, unless that breaks the budget
            const int last = tb.ext[pr.d - 1];
            int pitch = last;
            if (pr.d >= 2) {
                const int want = pr.d == 2 ? 16 : 8;
                int padded = last;
                while (padded % 32 != want) ++padded;
                if (elems * (size_t)padded * elt_b <= budget) pitch = padded;
            }
            tb.pad = pitch;
            elems *= (size_t)pitch;
            if (elems * elt_b > budget) ok = false;
            tb.use_lds = ok ? 1 : 0;
            if (ok) p->tile_elems = std::max<int>(p->tile_elems, (int)elems);
            return tb;
        };
        // adjoint lists: separable nodes in box form when their footprint fits
        // a class (the transposed row then scatters 3 L^2 (2D) entries instead
        // of 12 per landing point), the others per landing point
        if (p->opt.ckpt_every > 0) {
            // 2D: footprints up to 6 nodes; wider ones scatter faster per point
            // (measured: the box form's vector building and L^2 gathers cost
            // more than the FP64 LDS atomics they save from L = 8 on)
            static const int kLA[2][fk::kBoxClasses] = {{4, 6, 0, 0, 0}, {3, 4, 5, 6, 8}};
            const bool abox = node_ok && affine && p->d >= 2 && fk::box_compiled(p->d, p->qs) &&
                              sk != 1 && sk != 2;
            std::vector<std::vector<fk::WorkItem>> abw(fk::kBoxClasses);
            for (int i = 0; i < p->n_inst; ++i) {
                const fk_problem &pr = p->probs[i];
                int ac = -1;
                if (abox)
                    for (int c2 = 0; c2 < fk::kBoxClasses && ac < 0; ++c2)
                        if (inst_lneed[i] <= kLA[p->d - 2][c2]) ac = c2;
                std::vector<int> fw = inst_rest[i];
                if (ac < 0) {
                    fw.insert(fw.end(), inst_sep[i].begin(), inst_sep[i].end());
                } else {
                    std::vector<int> sep = inst_sep[i];
                    patch_sort(sep, pr, keys);
                    const int f0 = (int)p->adj.box_nodes.size();
                    p->adj.box_nodes.insert(p->adj.box_nodes.end(), sep.begin(), sep.end());
                    patch_work(abw[ac], i, keys, f0, kBlock);
                }
                patch_sort(fw, pr, keys);
                const int f1 = (int)p->adj.fw_nodes.size();
                p->adj.fw_nodes.insert(p->adj.fw_nodes.end(), fw.begin(), fw.end());
                patch_work(p->adj.fw_work, i, keys, f1, kBlock);
            }
            // 2D: work items none of whose nodes has a landing point that can
            // exit go first (their kernel has no exit tests)
            if (p->d == 2) {
                std::vector<fk::WorkItem> in, rest;
                for (fk::WorkItem it : p->adj.fw_work) {
                    bool all = true;
                    for (int u = 0; u < it.count && all; ++u)
                        all = inst_inner[it.inst][p->adj.fw_nodes[it.first + u]] != 0;
                    it.kind = all ? 1 : 0;
                    (all ? in : rest).push_back(it);
                }
                p->adj.n_in_work = (int)in.size();
                in.insert(in.end(), rest.begin(), rest.end());
                p->adj.fw_work.swap(in);
            }
            for (int c2 = 0; c2 < fk::kBoxClasses; ++c2) {
                p->adj.box_work_off[c2] = (int)p->adj.box_work.size();
                p->adj.n_box_work[c2] = (int)abw[c2].size();
                p->adj.box_work.insert(p->adj.box_work.end(), abw[c2].begin(), abw[c2].end());
            }
            for (const fk::WorkItem &it : p->adj.fw_work)
                p->adj.fw_tiles.push_back(tile_of(it, p->adj.fw_nodes, false));
            for (const fk::WorkItem &it : p->adj.box_work)
                // the box kernels index their tiles with unwrapped indices
                p->adj.box_tiles.push_back(tile_of(it, p->adj.box_nodes, true));
            stage_tiles(p);
        }
    }
    p->slope_work = tables;
    p->slope_work.insert(p->slope_work.end(), runs.begin(), runs.end());
    p->n_table_work = (int)tables.size();

    // per-(step, instance) time factors
    p->tfac.assign((size_t)p->N * p->n_inst * fk::kTimeFactors, 0.0);
    for (int n = 0; n < p->N; ++n) {
        const double t = p->t0 + (double)n * p->dt;
        for (int i = 0; i < p->n_inst; ++i) {
            const fk_problem &pr = p->probs[i];
            double *tf = &p->tfac[((size_t)n * p->n_inst + i) * fk::kTimeFactors];
            if (pr.coef_kind == FK_COEF_CELLULAR2D) {
                tf[0] = pr.coef[1] * std::sin(pr.coef[2] * t);
                tf[1] = std::sin(pr.coef[2] * t);
                tf[2] = std::cos(pr.coef[2] * t);
                tf[3] = t;
            } else if (pr.coef_kind == FK_COEF_RUNAWAY3D) {
                runaway_time_factors(pr, t, tf);
            } else if (pr.coef_kind == FK_COEF_ROLLS2D) {
                tf[0] = pr.coef[1] * std::cos(pr.coef[2] * t);
                tf[1] = std::cos(pr.coef[2] * t);
                tf[2] = std::sin(pr.coef[2] * t);
                tf[3] = t;
            } else if (pr.coef_kind == FK_COEF_ABC3D) {
                tf[0] = 1.0 + pr.coef[3] * std::sin(t);
                tf[1] = std::sin(t);
                tf[3] = t;
            } else {
                tf[3] = t;
            }
        }
    }

    if (p->opt.form == FK_FORM_ELL) {
        for (int a = 0; a < p->d; ++a)
            for (int i = 0; i < p->n_inst; ++i)
                if (p->probs[i].ax[a].periodic)
                    return fail(FK_ERR_UNSUPPORTED, "ELL form needs non-periodic axes");
        for (int a = 0; a < p->d; ++a) p->ell_box[a] = box[a];
        const long long W = ell_wmax;
        if (W * (long long)(kBlock / p->G) * 8 > 64 * 1024)   // FP64 row boxes in LDS
            return fail(FK_ERR_UNSUPPORTED, "ELL row box too large for LDS (%lld entries)", W);
        p->ell_width = (int)W;
        p->ell_total = ell_total;
        p->ell_entries = ell_rows_w;
        // width classes: bounds 128, 256, ... entries, the last one the widest row
        int bound[fk::kEllClasses];
        int nc = 0;
        for (long long bnd = 128; nc < fk::kEllClasses - 1 && bnd < W; bnd *= 2) bound[nc++] = (int)bnd;
        bound[nc++] = (int)W;
        // separable rows go to the direct (outer-product) assembly in runs of
        // up to 64 consecutive rows; the others to the LDS-box assembly in
        // runs of up to block / G rows
        std::vector<fk::WorkItem> rest_work;
        p->ell_sep_work.clear();
        p->ell_lmax = 1;
        for (int a = 0; a < p->d; ++a) p->ell_lmax = std::max(p->ell_lmax, p->ell_box[a]);
        // its per-thread axis vectors (d x 2 x lmax, 64 rows, and a zero column)
        // and the block table of an instance (16 bytes per block) must fit the
        // LDS; the table's column indices are bytes
        const bool f32e = p->opt.precision == FK_PREC_F32;
        const int ke = f32e ? 4 : 2;
        auto sep_table = [&](int i) { return (size_t)(p->d + 1) * (p->inst[i].ell_nbp / ke) * 16; };
        size_t tb_all = 0;
        for (int i = 0; i < p->n_inst; ++i) tb_all = std::max(tb_all, sep_table(i));
        const int zcol = p->d * 2 * p->ell_lmax;
        const bool sep_ok = zcol <= 255 &&
                            (size_t)(zcol + 1) * 64 * (f32e ? 4 : 8) + tb_all <= 60 * 1024;
        const int npb_e = kBlock / p->G;
        for (int i = 0; i < p->n_inst; ++i) {
            const std::vector<unsigned char> &sr = inst_seprow[i];
            const int na_i = (int)sr.size();
            for (int r = 0; r < na_i;) {
                const unsigned char sv = sr[r] && sep_ok;
                int e = r;
                while (e < na_i && (sr[e] && sep_ok) == (bool)sv) ++e;
                const int cap = sv ? 64 : npb_e;
                for (int f0 = r; f0 < e; f0 += cap) {
                    fk::WorkItem it;
                    std::memset(&it, 0, sizeof(it));
                    it.inst = i;
                    it.first = f0;
                    it.count = std::min(cap, e - f0);
                    (sv ? p->ell_sep_work : rest_work).push_back(it);
                }
                r = e;
            }
        }
        // separable runs by the instance's longest box axis (8, 16, 32, ...):
        // one launch per class, its LDS vectors sized by the class
        {
            std::vector<fk::WorkItem> sw;
            sw.swap(p->ell_sep_work);
            int nsc = 0;
            for (int lb = 8; nsc < fk::kEllClasses; lb *= 2) {
                const int lo = nsc == 0 ? 0 : lb / 2;
                int lmax_c = 0, first = (int)p->ell_sep_work.size();
                size_t tb_c = 0;
                for (const fk::WorkItem &it : sw) {
                    int li = 1;
                    for (int a = 0; a < p->d; ++a) li = std::max(li, p->inst[it.inst].ell_box[a]);
                    if (li > lo && li <= lb) {
                        p->ell_sep_work.push_back(it);
                        lmax_c = std::max(lmax_c, li);
                        tb_c = std::max(tb_c, sep_table(it.inst));
                    }
                }
                const int cnt = (int)p->ell_sep_work.size() - first;
                if (cnt > 0) {
                    p->ell_sep_off[nsc] = first;
                    p->ell_sep_n[nsc] = cnt;
                    p->ell_sep_l[nsc] = lmax_c;
                    p->ell_sep_tb[nsc] = (int)tb_c;
                    ++nsc;
                }
                if (lb >= p->ell_lmax) break;
            }
            p->n_ell_sep_cls = nsc;
        }
        std::vector<std::vector<fk::WorkItem>> by(nc);
        for (const fk::WorkItem &it : rest_work) {
            const int w = p->inst[it.inst].ell_w;
            int c = 0;
            while (bound[c] < w) ++c;
            by[c].push_back(it);
        }
        p->ell_work.clear();
        p->n_ell_cls = 0;
        for (int c = nc - 1; c >= 0; --c) {   // widest class first
            if (by[c].empty()) continue;
            const int k = p->n_ell_cls++;
            p->ell_cls_off[k] = (int)p->ell_work.size();
            p->ell_cls_n[k] = (int)by[c].size();
            int wmax = 0;
            for (const fk::WorkItem &it : by[c]) wmax = std::max(wmax, p->inst[it.inst].ell_w);
            p->ell_cls_w[k] = wmax;
            p->ell_work.insert(p->ell_work.end(), by[c].begin(), by[c].end());
        }
        // (the product keeps the instance order: sorted by width, the XCDs'
        // contiguous shares of one launch would be far from equal in work)
    }

    // workspace layout
    p->ws_bytes = 0;
    add_region(p, "inst", sizeof(fk::DevInst) * p->inst.size());
    add_region(p, "coords", sizeof(double) * p->coords.size());
    add_region(p, "active", sizeof(int) * std::max<size_t>(p->active.size(), 1));
    add_region(p, "cls", p->cls.size());
    add_region(p, "gh_a", sizeof(double) * p->gh_a.size());
    add_region(p, "gh_w", sizeof(double) * p->gh_w.size());
    add_region(p, "gh_wf", sizeof(float) * p->gh_wf.size());
    add_region(p, "gh_w1", sizeof(double) * p->gh_w1.size());
    add_region(p, "gh_w1f", sizeof(float) * p->gh_w1f.size());
    add_region(p, "tfac", sizeof(double) * p->tfac.size());
    add_region(p, "trig", sizeof(double) * 2 * std::max<size_t>(p->coords.size(), 1));
    add_region(p, "slope_work", sizeof(fk::WorkItem) * std::max<size_t>(p->slope_work.size(), 1));
    add_region(p, "node_work", sizeof(fk::WorkItem) * std::max<size_t>(p->node_work.size(), 1));
    add_region(p, "act_work", sizeof(fk::WorkItem) * std::max<size_t>(p->act_work.size(), 1));
    add_region(p, "ell_work", sizeof(fk::WorkItem) * std::max<size_t>(p->ell_work.size(), 1));
    add_region(p, "ell_sep_work", sizeof(fk::WorkItem) * std::max<size_t>(p->ell_sep_work.size(), 1));
    add_region(p, "row_work", sizeof(fk::WorkItem) * std::max<size_t>(p->row_work.size(), 1));
    add_region(p, "split_work", sizeof(fk::WorkItem) * std::max<size_t>(p->split_work.size(), 1));
    add_region(p, "afw_nodes", sizeof(int) * std::max<size_t>(p->adj.fw_nodes.size(), 1));
    add_region(p, "afw_work", sizeof(fk::WorkItem) * std::max<size_t>(p->adj.fw_work.size(), 1));
    add_region(p, "afw_tiles", sizeof(fk::TileBox) * std::max<size_t>(p->adj.fw_tiles.size(), 1));
    add_region(p, "abox_nodes", sizeof(int) * std::max<size_t>(p->adj.box_nodes.size(), 1));
    add_region(p, "abox_work", sizeof(fk::WorkItem) * std::max<size_t>(p->adj.box_work.size(), 1));
    add_region(p, "abox_tiles", sizeof(fk::TileBox) * std::max<size_t>(p->adj.box_tiles.size(), 1));
    add_region(p, "fw_nodes", sizeof(int) * std::max<size_t>(p->fw_nodes.size(), 1));
    add_region(p, "fw_work", sizeof(fk::WorkItem) * std::max<size_t>(p->fw_work.size(), 1));
    add_region(p, "fw_split_work", sizeof(fk::WorkItem) * std::max<size_t>(p->fw_split_work.size(), 1));
    add_region(p, "box_nodes", sizeof(int) * std::max<size_t>(p->box_nodes.size(), 1));
    add_region(p, "box_work", sizeof(fk::WorkItem) * std::max<size_t>(p->box_work.size(), 1));
    add_region(p, "flags", 64);
    const size_t fb = elt(p) * (size_t)p->n_nodes;
    add_region(p, "uA", fb);
    add_region(p, "uB", fb);
    add_region(p, "packed", fb * rec_stride(p->d));
    if (p->opt.hermite == FK_HERMITE_R2 && p->d == 3) add_region(p, "packed2", fb * 4);
    if (p->opt.form == FK_FORM_ELL) {
        const int nc = std::max(1, std::min(4, p->opt.columns));
        add_region(p, "packed_mc", fb * rec_stride(p->d) * nc);
        add_region(p, "ell_org", sizeof(int) * 3 * (size_t)std::max<long long>(p->n_active, 1));
        add_region(p, "ell_vals", elt(p) * (size_t)std::max<long long>(p->ell_total, 1));
        add_region(p, "ell_em", elt(p) * (size_t)std::max<long long>(p->n_active, 1));
    }
    p->ws_fwd_bytes = p->ws_bytes;   // tables, fields and records of the forward pass
    if (p->opt.ckpt_every > 0) {
        const int K = p->opt.ckpt_every;
        p->n_ckpt = (p->N - 1) / K + 2;
        add_region(p, "lamA", fb);
        add_region(p, "lamB", fb);
        add_region(p, "mu", fb * rec_stride(p->d));
        add_region(p, "stage", elt(p) * (size_t)std::max<long long>(p->adj.stage_entries, 1));
        add_region(p, "cov_node", sizeof(int) * std::max<size_t>(p->adj.cov_node.size(), 1));
        add_region(p, "cov_ptr", sizeof(int) * std::max<size_t>(p->adj.cov_ptr.size(), 1));
        add_region(p, "cov_base", sizeof(int) * std::max<size_t>(p->adj.cov_base.size(), 1));
        add_region(p, "grad", sizeof(double) * fk::kThetaSlots * p->n_inst);
        add_region(p, "ckpt", fb * p->n_ckpt);
        add_region(p, "seg", fb * std::max(1, std::min(K, p->N) - 1));   // recomputed fields
    }
    return FK_OK;
}

void fill_dev(fk_plan *p)
{
    fk::PlanDev &D = p->dev;
    std::memset(&D, 0, sizeof(D));
    D.inst = (const fk::DevInst *)p->at("inst");
    D.coords = (const double *)p->at("coords");
    D.active = (const int *)p->at("active");
    D.chi = (const unsigned char *)p->at("cls");
    D.gh_a = (const double *)p->at("gh_a");
    D.gh_w = (const double *)p->at("gh_w");
    D.gh_wf = (const float *)p->at("gh_wf");
    D.gh_w1 = (const double *)p->at("gh_w1");
    D.gh_w1f = (const float *)p->at("gh_w1f");
    D.tfac = (const double *)p->at("tfac");
    D.trig = (double2 *)p->at("trig");
    D.slope_work = (const fk::WorkItem *)p->at("slope_work");
    D.node_work = (const fk::WorkItem *)p->at("node_work");
    D.act_work = (const fk::WorkItem *)p->at("act_work");
    D.ell_work = (const fk::WorkItem *)p->at("ell_work");
    D.ell_sep_work = (const fk::WorkItem *)p->at("ell_sep_work");
    D.n_ell_sep_cls = p->n_ell_sep_cls;
    for (int c = 0; c < fk::kEllClasses; ++c) {
        D.ell_sep_off[c] = p->ell_sep_off[c];
        D.ell_sep_n[c] = p->ell_sep_n[c];
        D.ell_sep_l[c] = p->ell_sep_l[c];
        D.ell_sep_tb[c] = p->ell_sep_tb[c];
        // 256 threads share 64 rows; every workgroup resident at once
        int pc = 8;
        if (p->ell_sep_n[c] > 0)
            (void)fk::ell_per_cu(p->d, 1, p->f32, true,
                                 fk::ell_sep_lds(p->d, p->ell_sep_l[c], p->ell_sep_tb[c], p->f32), &pc);
        D.ell_sep_grid[c] = grid_for(p->ell_sep_n[c], pc);
    }
    D.n_ell_cls = p->n_ell_cls;
    for (int c = 0; c < fk::kEllClasses; ++c) {
        D.ell_cls_off[c] = p->ell_cls_off[c];
        D.ell_cls_n[c] = p->ell_cls_n[c];
        D.ell_cls_w[c] = p->ell_cls_w[c];
        int pc = 8;
        if (p->ell_cls_n[c] > 0)
            (void)fk::ell_per_cu(p->d, p->G, p->f32, false,
                                 (size_t)(kBlock / p->G) * p->ell_cls_w[c] * sizeof(double), &pc);
        D.ell_cls_grid[c] = grid_for(p->ell_cls_n[c], pc);
    }
    D.row_work = (const fk::WorkItem *)p->at("row_work");
    D.split_work = (const fk::WorkItem *)p->at("split_work");
    D.adj.fw_nodes = (const int *)p->at("afw_nodes");
    D.adj.fw_work = (const fk::WorkItem *)p->at("afw_work");
    D.adj.fw_tiles = (const fk::TileBox *)p->at("afw_tiles");
    D.adj.n_in_work = p->adj.n_in_work;
    D.adj.n_fw_work = (int)p->adj.fw_work.size() - p->adj.n_in_work;
    D.adj.in_grid = grid_for(p->adj.n_in_work);
    D.adj.fw_grid = grid_for(D.adj.n_fw_work);
    D.adj.box_nodes = (const int *)p->at("abox_nodes");
    D.adj.box_work = (const fk::WorkItem *)p->at("abox_work");
    D.adj.box_tiles = (const fk::TileBox *)p->at("abox_tiles");
    const bool staged = p->opt.ckpt_every > 0 && p->adj.stage_entries > 0;
    D.adj.stage = staged ? p->at("stage") : nullptr;
    D.adj.n_cov = staged ? (int)p->adj.cov_node.size() : 0;
    D.adj.cov_node = staged ? (const int *)p->at("cov_node") : nullptr;
    D.adj.cov_ptr = staged ? (const int *)p->at("cov_ptr") : nullptr;
    D.adj.cov_base = staged ? (const int *)p->at("cov_base") : nullptr;
    for (int c2 = 0; c2 < fk::kBoxClasses; ++c2) {
        D.adj.box_work_off[c2] = p->adj.box_work_off[c2];
        D.adj.n_box_work[c2] = p->adj.n_box_work[c2];
        D.adj.box_grid[c2] = grid_for(p->adj.n_box_work[c2]);
    }
    D.fw_nodes = (const int *)p->at("fw_nodes");
    D.fw_work = (const fk::WorkItem *)p->at("fw_work");
    D.n_fw_work = (int)p->fw_work.size();
    D.fw_grid = grid_for(p->fw_work.size());
    D.fw_split_work = (const fk::WorkItem *)p->at("fw_split_work");
    D.n_fw_split_work = (int)p->fw_split_work.size();
    D.fw_split_grid = grid_for(p->fw_split_work.size());
    D.box_nodes = (const int *)p->at("box_nodes");
    D.box_work = (const fk::WorkItem *)p->at("box_work");
    for (int c2 = 0; c2 < fk::kBoxClasses; ++c2) {
        D.box_work_off[c2] = p->box_work_off[c2];
        D.n_box_work[c2] = p->n_box_work[c2];
        D.box_grid[c2] = grid_for(p->n_box_work[c2]);
    }
    D.tile_elems = p->tile_elems;
    D.n_split_work = (int)p->split_work.size();
    D.split_grid = grid_for(p->split_work.size());
    D.flags = (int *)p->at("flags");
    D.n_inst = p->n_inst;
    D.n_slope_work = (int)p->slope_work.size();
    D.n_table_work = p->n_table_work;
    D.n_node_work = (int)p->node_work.size();
    D.n_act_work = (int)p->act_work.size();
    D.n_row_work = (int)p->row_work.size();
    D.d = p->d;
    D.qs = p->qs;
    D.n_quad = p->Q;
    D.n_steps = p->N;
    D.block = kBlock;
    D.group = p->G;
    D.hermite2 = (p->opt.hermite == FK_HERMITE_R2 && p->d >= 2) ? 1 : 0;
    D.packed2 = (p->opt.hermite == FK_HERMITE_R2 && p->d == 3) ? p->at("packed2") : nullptr;
    D.faces = p->faces ? 1 : 0;
    D.all_affine = 1;
    for (const fk::DevInst &I : p->inst)
        for (int a = 0; a < p->d; ++a)
            if (!I.affine[a]) D.all_affine = 0;
    D.step_kind = p->step_kind;
    D.slope_grid = grid_for(p->slope_work.size());
    D.node_grid = grid_for(p->node_work.size());
    D.act_grid = grid_for(p->act_work.size());
    D.row_grid = grid_for(p->row_work.size());
    D.dt = p->dt;
    D.t0 = p->t0;
    D.n_nodes = p->n_nodes;
    D.n_active = p->n_active;
    D.ell_width = p->ell_width;
    for (int a = 0; a < 3; ++a) D.ell_box[a] = p->ell_box[a];
    D.ell_grid = D.act_grid;
}

fk_status need_ws(const fk_plan *p)
{
    if (!p) return fail(FK_ERR_ARG, "null plan");
    if (!p->ws) return fail(FK_ERR_STATE, "no workspace set (fk_plan_set_workspace)");
    return FK_OK;
}

#define FK_TRY(expr)                         \
    do {                                     \
        fk_status s_ = (expr);               \
        if (s_ != FK_OK) return s_;          \
    } while (0)

#define FK_LAUNCH(expr)                                                               \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(FK_ERR_HIP, "launch failed: %s", hipGetErrorString(e_));     \
    } while (0)

// One step u_next -> u_out (u_out must hold 1 on exit nodes already).
fk_status enqueue_step(fk_plan *p, int n, const void *u_next, void *u_out, hipStream_t s)
{
    void *packed = p->at("packed");
    FK_LAUNCH(fk::launch_slopes(p->dev, p->f32, n, u_next, packed, s));
    if (p->opt.form == FK_FORM_ELL) {
        int *cols = (int *)p->at("ell_org");
        void *vals = p->at("ell_vals"), *em = p->at("ell_em");
        FK_LAUNCH(fk::launch_assemble_ell(p->dev, p->f32, n, cols, vals, em, s));
        FK_LAUNCH(fk::launch_ell_apply(p->dev, p->f32, cols, vals, em, packed, u_out, s));
    } else {
        FK_LAUNCH(fk::launch_step_fused(p->dev, p->f32, n, packed, u_out, s));
    }
    return FK_OK;
}

// Backward loop from u_start (a field at step `start`) down to step 0,
// copying snapshots.  ckpt: optional checkpoint store (adjoint).
fk_status enqueue_pass(fk_plan *p, const void *u_start, int start, const int *snaps, int n_snap,
                       void *u_out, hipStream_t s, bool store_ckpt)
{
    const size_t fb = elt(p) * (size_t)p->n_nodes;
    void *ua = p->at("uA"), *ub = p->at("uB");
    FK_LAUNCH(fk::launch_clear_flags(p->dev, s));
    // both buffers hold 1 on exit nodes (and chi elsewhere)
    FK_LAUNCH(fk::launch_init_field(p->dev, p->f32, ub, s));
    if (u_start && p->conv) {
        FK_LAUNCH(fk::launch_convert_in(p->dev, (const float *)u_start, (double *)ua, s));
    } else if (u_start) {
        FK_HIP(hipMemcpyAsync(ua, u_start, fb, hipMemcpyDeviceToDevice, s));
    } else {
        FK_LAUNCH(fk::launch_init_field(p->dev, p->f32, ua, s));
    }
    auto snap_copy = [&](int n, const void *u) -> fk_status {
        for (int k = 0; k < n_snap; ++k) {
            if (snaps[k] != n) continue;
            if (p->conv)
                FK_LAUNCH(fk::launch_convert_out(p->dev, (const double *)u,
                                                 (float *)u_out + (size_t)k * p->out_n_nodes, s));
            else
                FK_HIP(hipMemcpyAsync((unsigned char *)u_out + (size_t)k * fb, u, fb,
                                      hipMemcpyDeviceToDevice, s));
        }
        return FK_OK;
    };
    auto ckpt_copy = [&](int n, const void *u) -> fk_status {
        if (!store_ckpt) return FK_OK;
        const int K = p->opt.ckpt_every;
        int slot = -1;
        if (n == p->N) slot = p->n_ckpt - 1;
        else if (n % K == 0) slot = n / K;
        if (slot >= 0)
            FK_HIP(hipMemcpyAsync((unsigned char *)p->at("ckpt") + (size_t)slot * fb, u, fb,
                                  hipMemcpyDeviceToDevice, s));
        return FK_OK;
    };
    FK_TRY(snap_copy(start, ua));
    FK_TRY(ckpt_copy(start, ua));
    // a step whose state is a checkpoint writes it straight into its slot
    // (the slots hold 1 on exit nodes since the workspace was set); the others
    // alternate between the two work fields
    auto slot_of = [&](int n) -> void * {
        if (!store_ckpt || n == p->N || n % p->opt.ckpt_every != 0) return nullptr;
        return (unsigned char *)p->at("ckpt") + (size_t)(n / p->opt.ckpt_every) * fb;
    };
    void *cur = ua;
    for (int n = start - 1; n >= 0; --n) {
        void *dst = slot_of(n);
        if (!dst) dst = (cur == ua) ? ub : ua;
        FK_TRY(enqueue_step(p, n, cur, dst, s));
        cur = dst;
        FK_TRY(snap_copy(n, cur));
    }
    return FK_OK;
}

// Runs body on s, captured once into a HIP graph and replayed while key
// (the body's arguments) stays the same, when the plan uses graphs.
template <typename Body>
fk_status run_captured(fk_plan *p, const std::string &k, hipStream_t s, const Body &body)
{
    if (!p->opt.use_graph) return body(s);
    if (!p->gexec || k != p->gkey) {
        if (p->gexec) {
            (void)hipGraphExecDestroy(p->gexec);
            p->gexec = nullptr;
        }
        if (!p->cap_stream) FK_HIP(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        FK_HIP(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
        fk_status st = body(p->cap_stream);
        hipError_t e = hipStreamEndCapture(p->cap_stream, &graph);
        if (st != FK_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) return fail(FK_ERR_HIP, "graph capture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&p->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return fail(FK_ERR_HIP, "graph instantiate: %s", hipGetErrorString(e));
        p->gkey = k;
    }
    FK_HIP(hipGraphLaunch(p->gexec, s));
    return FK_OK;
}

fk_status run_pass(fk_plan *p, const void *u_start, int start, const int *snaps, int n_snap,
                   void *u_out, hipStream_t s, bool store_ckpt)
{
    char key[256];
    snprintf(key, sizeof(key), "pass|%p|%d|%p|%d|", u_start, start, u_out, store_ckpt ? 1 : 0);
    std::string k = key;
    for (int i = 0; i < n_snap; ++i) k += std::to_string(snaps[i]) + ",";
    return run_captured(p, k, s, [&](hipStream_t cs) {
        return enqueue_pass(p, u_start, start, snaps, n_snap, u_out, cs, store_ckpt);
    });
}

// Algorithm 1: columns u_out[h] (in place), sweep index n = M .. 1 with the
// operator of step n - 1 shared by the columns whose horizon is >= n.
fk_status enqueue_horizons(fk_plan *p, const int *hz, int n_h, void *u_out, hipStream_t s)
{
    const size_t fe = (size_t)p->n_nodes;              // elements per field
    const size_t fb = elt(p) * fe;
    std::vector<int> order(n_h);
    for (int h = 0; h < n_h; ++h) order[h] = h;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return hz[a] < hz[b]; });
    int M = 0;
    for (int h = 0; h < n_h; ++h) M = std::max(M, hz[h]);
    auto col = [&](int h) { return (void *)((unsigned char *)u_out + (size_t)h * fb); };
    FK_LAUNCH(fk::launch_clear_flags(p->dev, s));
    for (int h = 0; h < n_h; ++h) FK_LAUNCH(fk::launch_init_field(p->dev, p->f32, col(h), s));
    const bool ell = p->opt.form == FK_FORM_ELL;
    const int chunk = std::max(1, std::min(4, p->opt.columns));
    void *packed = p->at("packed");
    size_t first = order.size();   // order[first ..] are the columns with horizon >= n
    for (int n = M; n >= 1; --n) {
        while (first > 0 && hz[order[first - 1]] >= n) --first;
        const int step = n - 1;
        if (!ell) {
            for (size_t k = first; k < order.size(); ++k) {
                FK_LAUNCH(fk::launch_slopes(p->dev, p->f32, step, col(order[k]), packed, s));
                FK_LAUNCH(fk::launch_step_fused(p->dev, p->f32, step, packed, col(order[k]), s));
            }
            continue;
        }
        int *org = (int *)p->at("ell_org");
        void *vals = p->at("ell_vals"), *em = p->at("ell_em");
        unsigned char *planes = (unsigned char *)p->at("packed_mc");
        const size_t plane_b = fb * rec_stride(p->d);
        FK_LAUNCH(fk::launch_tables(p->dev, step, s));
        FK_LAUNCH(fk::launch_assemble_ell(p->dev, p->f32, step, org, vals, em, s));
        for (size_t k0 = first; k0 < order.size();) {
            // columns of consecutive storage in one launch: runs of order[]
            // entries whose fields are adjacent in u_out
            int nc = 1;
            while (nc < chunk && k0 + nc < order.size() && order[k0 + nc] == order[k0] + nc) ++nc;
            for (int c = 0; c < nc; ++c)
                FK_LAUNCH(fk::launch_slopes(p->dev, p->f32, step, col(order[k0 + c]),
                                            planes + (size_t)c * plane_b, s));
            FK_LAUNCH(fk::launch_ell_apply_mc(p->dev, p->f32, org, vals, em, planes,
                                              (long long)(fe * rec_stride(p->d)), col(order[k0]),
                                              (long long)fe, nc, s));
            k0 += nc;
        }
    }
    return FK_OK;
}

// Copies the plan's host tables into the workspace the plan points at
// (asynchronous on s) and clears the device flags.
fk_status upload_tables(fk_plan *p, hipStream_t s);

fk_status check_snaps(const fk_plan *p, const int *snaps, int n_snap, int start, const void *u_out)
{
    if (n_snap < 0) return fail(FK_ERR_ARG, "n_snap < 0");
    if (n_snap > 0 && (!snaps || !u_out)) return fail(FK_ERR_ARG, "null snapshot list or output");
    for (int k = 0; k < n_snap; ++k)
        if (snaps[k] < 0 || snaps[k] > start)
            return fail(FK_ERR_ARG, "snapshot step %d outside [0, %d]", snaps[k], start);
    (void)p;
    return FK_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *fk_last_error(void) { return g_err.c_str(); }

int fk_version(void) { return FK_ABI_VERSION; }

fk_status fk_gh_rule(int q, double *nodes, double *weights)
{
    return gh_rule_impl(q, nodes, weights);
}

fk_status fk_plan_create(const fk_problem *probs, int n_inst, const fk_options *opt, fk_plan **out)
{
    g_err.clear();
    if (!out) return fail(FK_ERR_ARG, "null output plan pointer");
    *out = nullptr;
    if (!probs || n_inst < 1) return fail(FK_ERR_ARG, "need n_inst >= 1 problems");
    fk_options o{};
    if (opt) o = *opt;
    if (o.precision != FK_PREC_F64 && o.precision != FK_PREC_F32)
        return fail(FK_ERR_ARG, "precision must be FK_PREC_F64 or FK_PREC_F32");
    if (o.form != FK_FORM_FUSED && o.form != FK_FORM_ELL)
        return fail(FK_ERR_ARG, "form must be FK_FORM_FUSED or FK_FORM_ELL");
    if (o.ckpt_every < 0) return fail(FK_ERR_ARG, "ckpt_every must be >= 0");
    if (o.block != 0 && o.block != kBlock) return fail(FK_ERR_UNSUPPORTED, "block must be 0 or 256");
    if (o.step_kernel < 0 || o.step_kernel > 4) return fail(FK_ERR_ARG, "step_kernel must be 0..4");
    if (o.columns < 0 || o.columns > 4) return fail(FK_ERR_ARG, "columns must be 0..4");
    if (o.hermite != FK_HERMITE_R1 && o.hermite != FK_HERMITE_R2)
        return fail(FK_ERR_ARG, "hermite must be FK_HERMITE_R1 or FK_HERMITE_R2");
    if (o.hermite == FK_HERMITE_R2) {
        if (o.form != FK_FORM_FUSED) return fail(FK_ERR_UNSUPPORTED, "the R2 interpolant needs the fused form");
        if (probs[0].d == 3) {
            // 3D: the twist records are read by the thread-per-node step only
            if (!fk::step_node_compiled(3, probs[0].gh_q))
                return fail(FK_ERR_UNSUPPORTED, "the 3D R2 interpolant needs a thread-per-node "
                            "kernel for gh_q=%d", probs[0].gh_q);
            if (o.step_kernel == 2 || o.step_kernel == 4)
                return fail(FK_ERR_UNSUPPORTED, "the 3D R2 interpolant runs in the "
                            "thread-per-node step");
            for (int i = 0; i < n_inst; ++i)
                for (int a = 0; a < 3; ++a)
                    if (probs[i].face[a][0] != FK_FACE_EXIT1 || probs[i].face[a][1] != FK_FACE_EXIT1 ||
                        probs[i].coef_kind == FK_COEF_RUNAWAY3D)
                        return fail(FK_ERR_UNSUPPORTED, "instance %d: the 3D R2 interpolant takes "
                                    "exit-1 faces only", i);
        }
        if (o.ckpt_every > 0) return fail(FK_ERR_UNSUPPORTED, "no adjoint of the R2 interpolant");
    }
    if ((o.step_kernel == 1 || o.step_kernel == 3 || o.step_kernel == 4) &&
        !fk::step_node_compiled(probs[0].d, probs[0].gh_q))
        return fail(FK_ERR_UNSUPPORTED, "no thread-per-node kernel compiled for d=%d, gh_q=%d",
                    probs[0].d, probs[0].gh_q);
    for (int i = 0; i < n_inst; ++i) FK_TRY(validate(probs[i], i));
    const fk_problem &a = probs[0];
    for (int i = 1; i < n_inst; ++i) {
        const fk_problem &b = probs[i];
        if (b.d != a.d || b.gh_q != a.gh_q || b.dt != a.dt || b.n_steps != a.n_steps ||
            b.t0 != a.t0 || b.coef_kind != a.coef_kind || b.region_kind != a.region_kind)
            return fail(FK_ERR_ARG, "instance %d: d, gh_q, dt, n_steps, t0, coef_kind and "
                        "region_kind must match instance 0", i);
    }
    for (int i = 0; i < n_inst; ++i) {
        bool fc = probs[i].coef_kind == FK_COEF_RUNAWAY3D;
        for (int a = 0; a < probs[i].d; ++a)
            fc = fc || probs[i].face[a][0] != FK_FACE_EXIT1 || probs[i].face[a][1] != FK_FACE_EXIT1;
        if (fc && (o.form != FK_FORM_FUSED || o.ckpt_every > 0))
            return fail(FK_ERR_UNSUPPORTED, "instance %d: face kinds other than exit-1 and the "
                        "runaway model run the fused forward calls only", i);
    }
    if (o.ckpt_every > 0)
        for (int i = 0; i < n_inst; ++i)
            if (!(probs[i].D > 0)) return fail(FK_ERR_ARG, "adjoint needs D > 0 (instance %d)", i);
    std::vector<int> forced;
    if (o.precision == FK_PREC_F32)
        for (int i = 0; i < n_inst; ++i)
            if (probs[i].force_f64) forced.push_back(i);
    if (!forced.empty() && o.form != FK_FORM_FUSED)
        return fail(FK_ERR_UNSUPPORTED, "instances forced to FP64 need the fused form");
    fk_plan *p = new (std::nothrow) fk_plan();
    if (!p) return fail(FK_ERR_ARG, "out of host memory");
    p->opt = o;
    p->f32 = o.precision == FK_PREC_F32;
    p->n_inst = n_inst;
    if (!forced.empty()) {
        p->skip.assign(n_inst, 0);
        for (int i : forced) p->skip[i] = 1;
    }
    p->probs.assign(probs, probs + n_inst);
    for (auto &pr : p->probs)
        for (int ax = 0; ax < 3; ++ax) pr.ax[ax].nodes = nullptr;   // copied into coords
    // build from the caller's arrays (still valid during this call)
    std::vector<fk_problem> tmp(probs, probs + n_inst);
    std::swap(p->probs, tmp);
    fk_status st = build_plan(p);
    std::swap(p->probs, tmp);
    if (st != FK_OK) {
        delete p;
        return st;
    }
    if (!forced.empty()) {
        std::vector<fk_problem> sp;
        for (int i : forced) {
            sp.push_back(probs[i]);
            sp.back().force_f64 = 0;
        }
        fk_options so = o;
        so.precision = FK_PREC_F64;
        fk_plan *c = nullptr;
        st = fk_plan_create(sp.data(), (int)sp.size(), &so, &c);
        if (st != FK_OK) {
            delete p;
            return st;
        }
        c->conv = true;
        c->out_n_nodes = p->n_nodes;
        c->parent_inst = forced;
        for (size_t k = 0; k < forced.size(); ++k) {
            c->inst[k].out_off = p->inst[forced[k]].node_off;
            p->act_count[forced[k]] = c->act_count[k];
        }
        p->sub = c;
        p->sub_inst = forced;
        add_region(p, "sub_ws", c->ws_bytes);
    }
    *out = p;
    return FK_OK;
}

void fk_plan_destroy(fk_plan *p)
{
    if (!p) return;
    fk_plan_destroy(p->sub);
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    delete p;
}

fk_status fk_plan_get_info(const fk_plan *p, fk_plan_info *info)
{
    if (!p || !info) return fail(FK_ERR_ARG, "null argument");
    info->n_inst = p->n_inst;
    info->d = p->d;
    info->gh_q = p->qs;
    info->n_quad = p->Q;
    info->n_steps = p->N;
    info->n_theta = p->n_theta;
    info->n_nodes = p->n_nodes;
    info->n_active = p->n_active;
    info->ell_width = p->ell_width;
    info->ell_entries = p->opt.form == FK_FORM_ELL ? p->ell_entries : 0;
    info->adj_point_nodes = (int64_t)p->adj.fw_nodes.size();
    info->adj_box_nodes = (int64_t)p->adj.box_nodes.size();
    info->workspace_bytes = p->ws_bytes;
    if (p->sub) {
        info->n_active += p->sub->n_active;
        info->adj_point_nodes += (int64_t)p->sub->adj.fw_nodes.size();
        info->adj_box_nodes += (int64_t)p->sub->adj.box_nodes.size();
    }
    return FK_OK;
}

fk_status fk_plan_layout(const fk_plan *p, int64_t *node_offset, int64_t *active_count)
{
    if (!p) return fail(FK_ERR_ARG, "null plan");
    if (node_offset)
        for (int i = 0; i <= p->n_inst; ++i) node_offset[i] = p->node_off[i];
    if (active_count)
        for (int i = 0; i < p->n_inst; ++i) active_count[i] = p->act_count[i];
    return FK_OK;
}

fk_status fk_plan_set_workspace(fk_plan *p, void *dev_ptr, size_t bytes, void *stream)
{
    if (!p) return fail(FK_ERR_ARG, "null plan");
    if (!dev_ptr) return fail(FK_ERR_ARG, "null workspace");
    if (((uintptr_t)dev_ptr) % kAlign) return fail(FK_ERR_ARG, "workspace must be 256-byte aligned");
    if (bytes < p->ws_bytes)
        return fail(FK_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", bytes, p->ws_bytes);
    hipStream_t s = (hipStream_t)stream;
    if (p->gexec) {
        (void)hipGraphExecDestroy(p->gexec);
        p->gexec = nullptr;
        p->gkey.clear();
    }
    p->ws = (unsigned char *)dev_ptr;
    p->ckpt_valid = false;
    fill_dev(p);
    FK_TRY(upload_tables(p, s));
    if (p->opt.ckpt_every > 0) {
        // checkpoint slots hold 1 on exit nodes for good: the forward pass
        // writes only the active nodes (and their images) of a slot
        const size_t fb = elt(p) * (size_t)p->n_nodes;
        for (int k = 0; k < p->n_ckpt; ++k)
            FK_LAUNCH(fk::launch_init_field(p->dev, p->f32, (unsigned char *)p->at("ckpt") + (size_t)k * fb, s));
    }
    FK_HIP(hipStreamSynchronize(s));
    if (p->sub) FK_TRY(fk_plan_set_workspace(p->sub, p->at("sub_ws"), p->sub->ws_bytes, stream));
    return FK_OK;
}

fk_status fk_forward_static(fk_plan *p, const int *snap_steps, int n_snap, void *u_out,
                            void *stream)
{
    if (!p) return fail(FK_ERR_ARG, "null plan");
    FK_TRY(check_snaps(p, snap_steps, n_snap, p->N, u_out));
    if (p->sub) return fail(FK_ERR_UNSUPPORTED, "plans with instances forced to FP64");
    if (p->ws_fwd_bytes > (size_t)FK_STATIC_SCRATCH_BYTES)
        return fail(FK_ERR_WORKSPACE,
                    "plan needs %zu bytes of forward workspace, the static scratch holds %zu",
                    p->ws_fwd_bytes, (size_t)FK_STATIC_SCRATCH_BYTES);
    void *scr = nullptr;
    hipError_t e = fk::static_scratch(&scr);
    if (e != hipSuccess) return fail(FK_ERR_HIP, "static scratch: %s", hipGetErrorString(e));
    hipStream_t s = (hipStream_t)stream;
    // run on the static scratch, then give the plan back its own workspace
    // (host-side pointers only: the caller's workspace is not touched)
    unsigned char *saved_ws = p->ws;
    const fk::PlanDev saved_dev = p->dev;
    p->ws = (unsigned char *)scr;
    fill_dev(p);
    fk_status st = upload_tables(p, s);
    if (st == FK_OK) st = enqueue_pass(p, nullptr, p->N, snap_steps, n_snap, u_out, s, false);
    p->ws = saved_ws;
    p->dev = saved_dev;
    return st;
}

}  // extern "C"

namespace {

fk_status upload_tables(fk_plan *p, hipStream_t s)
{
    auto up = [&](const char *name, const void *src, size_t n) -> fk_status {
        if (n) FK_HIP(hipMemcpyAsync(p->at(name), src, n, hipMemcpyHostToDevice, s));
        return FK_OK;
    };
    FK_TRY(up("inst", p->inst.data(), sizeof(fk::DevInst) * p->inst.size()));
    FK_TRY(up("coords", p->coords.data(), sizeof(double) * p->coords.size()));
    FK_TRY(up("active", p->active.data(), sizeof(int) * p->active.size()));
    FK_TRY(up("cls", p->cls.data(), p->cls.size()));
    FK_TRY(up("gh_a", p->gh_a.data(), sizeof(double) * p->gh_a.size()));
    FK_TRY(up("gh_w", p->gh_w.data(), sizeof(double) * p->gh_w.size()));
    FK_TRY(up("gh_wf", p->gh_wf.data(), sizeof(float) * p->gh_wf.size()));
    FK_TRY(up("gh_w1", p->gh_w1.data(), sizeof(double) * p->gh_w1.size()));
    FK_TRY(up("gh_w1f", p->gh_w1f.data(), sizeof(float) * p->gh_w1f.size()));
    FK_TRY(up("tfac", p->tfac.data(), sizeof(double) * p->tfac.size()));
    FK_TRY(up("slope_work", p->slope_work.data(), sizeof(fk::WorkItem) * p->slope_work.size()));
    FK_TRY(up("node_work", p->node_work.data(), sizeof(fk::WorkItem) * p->node_work.size()));
    FK_TRY(up("act_work", p->act_work.data(), sizeof(fk::WorkItem) * p->act_work.size()));
    FK_TRY(up("ell_work", p->ell_work.data(), sizeof(fk::WorkItem) * p->ell_work.size()));
    FK_TRY(up("ell_sep_work", p->ell_sep_work.data(), sizeof(fk::WorkItem) * p->ell_sep_work.size()));
    FK_TRY(up("row_work", p->row_work.data(), sizeof(fk::WorkItem) * p->row_work.size()));
    FK_TRY(up("split_work", p->split_work.data(), sizeof(fk::WorkItem) * p->split_work.size()));
    FK_TRY(up("afw_nodes", p->adj.fw_nodes.data(), sizeof(int) * p->adj.fw_nodes.size()));
    FK_TRY(up("afw_work", p->adj.fw_work.data(), sizeof(fk::WorkItem) * p->adj.fw_work.size()));
    FK_TRY(up("afw_tiles", p->adj.fw_tiles.data(), sizeof(fk::TileBox) * p->adj.fw_tiles.size()));
    FK_TRY(up("abox_nodes", p->adj.box_nodes.data(), sizeof(int) * p->adj.box_nodes.size()));
    FK_TRY(up("abox_work", p->adj.box_work.data(), sizeof(fk::WorkItem) * p->adj.box_work.size()));
    FK_TRY(up("abox_tiles", p->adj.box_tiles.data(), sizeof(fk::TileBox) * p->adj.box_tiles.size()));
    if (p->opt.ckpt_every > 0 && p->adj.stage_entries > 0) {
        FK_TRY(up("cov_node", p->adj.cov_node.data(), sizeof(int) * p->adj.cov_node.size()));
        FK_TRY(up("cov_ptr", p->adj.cov_ptr.data(), sizeof(int) * p->adj.cov_ptr.size()));
        FK_TRY(up("cov_base", p->adj.cov_base.data(), sizeof(int) * p->adj.cov_base.size()));
    }
    FK_TRY(up("fw_nodes", p->fw_nodes.data(), sizeof(int) * p->fw_nodes.size()));
    FK_TRY(up("fw_work", p->fw_work.data(), sizeof(fk::WorkItem) * p->fw_work.size()));
    FK_TRY(up("fw_split_work", p->fw_split_work.data(), sizeof(fk::WorkItem) * p->fw_split_work.size()));
    FK_TRY(up("box_nodes", p->box_nodes.data(), sizeof(int) * p->box_nodes.size()));
    FK_TRY(up("box_work", p->box_work.data(), sizeof(fk::WorkItem) * p->box_work.size()));
    FK_LAUNCH(fk::launch_clear_flags(p->dev, s));
    return FK_OK;
}

}  // namespace

extern "C" {

fk_status fk_forward(fk_plan *p, const int *snap_steps, int n_snap, void *u_out, void *stream)
{
    FK_TRY(need_ws(p));
    FK_TRY(check_snaps(p, snap_steps, n_snap, p->N, u_out));
    // a plan built for the adjoint stores its checkpoints on the way
    for (fk_plan *q = p; q; q = q->sub) {
        const bool store = q->opt.ckpt_every > 0;
        q->ckpt_valid = false;
        FK_TRY(run_pass(q, nullptr, q->N, snap_steps, n_snap, u_out, (hipStream_t)stream, store));
        q->ckpt_valid = store;
        q->ckpt_stream = (hipStream_t)stream;
    }
    return FK_OK;
}

fk_status fk_forward_horizons(fk_plan *p, const int *horizons, int n_h, void *u_out, void *stream)
{
    FK_TRY(need_ws(p));
    if (!horizons || n_h < 1 || !u_out) return fail(FK_ERR_ARG, "null horizons or output, or n_h < 1");
    for (int h = 0; h < n_h; ++h)
        if (horizons[h] < 1 || horizons[h] > p->N)
            return fail(FK_ERR_ARG, "horizon %d outside [1, %d]", horizons[h], p->N);
    if (p->sub) return fail(FK_ERR_UNSUPPORTED, "plans with instances forced to FP64");
    char key[64];
    snprintf(key, sizeof(key), "horizons|%p|", u_out);
    std::string k = key;
    for (int h = 0; h < n_h; ++h) k += std::to_string(horizons[h]) + ",";
    return run_captured(p, k, (hipStream_t)stream, [&](hipStream_t cs) {
        return enqueue_horizons(p, horizons, n_h, u_out, cs);
    });
}

fk_status fk_forward_from(fk_plan *p, const void *u_start, int start_step, const int *snap_steps,
                          int n_snap, void *u_out, void *stream)
{
    FK_TRY(need_ws(p));
    if (!u_start) return fail(FK_ERR_ARG, "null start state");
    if (start_step < 0 || start_step > p->N) return fail(FK_ERR_ARG, "start_step outside [0, N]");
    FK_TRY(check_snaps(p, snap_steps, n_snap, start_step, u_out));
    for (fk_plan *q = p; q; q = q->sub)
        FK_TRY(run_pass(q, u_start, start_step, snap_steps, n_snap, u_out, (hipStream_t)stream, false));
    return FK_OK;
}

fk_status fk_step(fk_plan *p, int n, const void *u_next, void *u_out, void *stream)
{
    FK_TRY(need_ws(p));
    if (!u_next || !u_out) return fail(FK_ERR_ARG, "null field");
    if (n < 0 || n >= p->N) return fail(FK_ERR_ARG, "step %d outside [0, N-1]", n);
    hipStream_t s = (hipStream_t)stream;
    FK_LAUNCH(fk::launch_init_field(p->dev, p->f32, u_out, s));
    FK_TRY(enqueue_step(p, n, u_next, u_out, s));
    if (fk_plan *c = p->sub) {
        double *ua = (double *)c->at("uA"), *ub = (double *)c->at("uB");
        FK_LAUNCH(fk::launch_convert_in(c->dev, (const float *)u_next, ua, s));
        FK_LAUNCH(fk::launch_init_field(c->dev, false, ub, s));
        FK_TRY(enqueue_step(c, n, ua, ub, s));
        FK_LAUNCH(fk::launch_convert_out(c->dev, ub, (float *)u_out, s));
    }
    return FK_OK;
}

fk_status fk_apply_step(fk_plan *p, int n, int transpose, const void *x, void *y, void *stream)
{
    FK_TRY(need_ws(p));
    if (!x || !y) return fail(FK_ERR_ARG, "null field");
    if (n < 0 || n >= p->N) return fail(FK_ERR_ARG, "step %d outside [0, N-1]", n);
    if (transpose && p->opt.ckpt_every <= 0)
        return fail(FK_ERR_STATE, "the transposed operator needs a plan created with ckpt_every > 0");
    if (p->sub) return fail(FK_ERR_UNSUPPORTED, "plans with instances forced to FP64");
    hipStream_t s = (hipStream_t)stream;
    const size_t fb = elt(p) * (size_t)p->n_nodes;
    void *packed = p->at("packed");
    // coefficient tables of step n (the slope pass is replaced by caller data)
    FK_LAUNCH(fk::launch_tables(p->dev, n, s));
    auto apply = [&](void *out) -> fk_status {
        FK_LAUNCH(fk::launch_init_field(p->dev, p->f32, out, s));
        if (p->opt.form == FK_FORM_ELL) {
            int *cols = (int *)p->at("ell_org");
            void *vals = p->at("ell_vals"), *em = p->at("ell_em");
            FK_LAUNCH(fk::launch_assemble_ell(p->dev, p->f32, n, cols, vals, em, s));
            FK_LAUNCH(fk::launch_ell_apply(p->dev, p->f32, cols, vals, em, packed, out, s));
        } else {
            FK_LAUNCH(fk::launch_step_fused(p->dev, p->f32, n, packed, out, s));
        }
        return FK_OK;
    };
    if (!transpose) {
        // the step kernels evaluate the affine map [u; g] -> A_n [u; g] + e
        // (e = exit mass); A_n x is that map at x minus the map at 0
        void *ya = p->at("uA"), *yb = p->at("uB");
        FK_LAUNCH(fk::launch_pack_fields(p->dev, p->f32, x, packed, s));
        FK_TRY(apply(ya));
        FK_LAUNCH(fk::launch_zero(packed, fb * rec_stride(p->d), s));
        FK_TRY(apply(yb));
        FK_LAUNCH(fk::launch_masked_diff(p->dev, p->f32, ya, yb, y, s));
    } else {
        // mu = A_n^T lam with lam = y on the active rows: the adjoint step's
        // scatter; its theta-gradient (zero records) goes to the plan's
        // gradient buffer and is discarded
        void *la = p->at("lamA"), *mu = p->at("mu");
        double *g = (double *)p->at("grad");
        FK_LAUNCH(fk::launch_zero(packed, fb * rec_stride(p->d), s));
        FK_LAUNCH(fk::launch_masked_diff(p->dev, p->f32, x, nullptr, la, s));
        FK_LAUNCH(fk::launch_zero(mu, fb * rec_stride(p->d), s));
        FK_LAUNCH(fk::launch_zero(g, sizeof(double) * fk::kThetaSlots * p->n_inst, s));
        FK_LAUNCH(fk::launch_adjoint_step(p->dev, p->f32, n, packed, la, mu, g, s));
        FK_LAUNCH(fk::launch_unpack_fields(p->dev, p->f32, mu, y, s));
        FK_LAUNCH(fk::launch_zero(mu, fb * rec_stride(p->d), s));
    }
    return FK_OK;
}

fk_status fk_export_cells(fk_plan *p, int inst, int n, int *cells, unsigned char *exit_flags,
                          void *stream)
{
    FK_TRY(need_ws(p));
    if (inst < 0 || inst >= p->n_inst) return fail(FK_ERR_ARG, "instance out of range");
    if (n < 0 || n >= p->N) return fail(FK_ERR_ARG, "step outside [0, N-1]");
    if (!cells || !exit_flags) return fail(FK_ERR_ARG, "null output");
    if (p->sub)
        for (size_t k = 0; k < p->sub_inst.size(); ++k)
            if (p->sub_inst[k] == inst) return fk_export_cells(p->sub, (int)k, n, cells, exit_flags, stream);
    FK_LAUNCH(fk::launch_tables(p->dev, n, (hipStream_t)stream));
    FK_LAUNCH(fk::launch_export_cells(p->dev, inst, n, cells, exit_flags, (hipStream_t)stream));
    return FK_OK;
}

fk_status fk_export_ell(fk_plan *p, int n, int *cols, void *vals, void *exit_mass, void *stream)
{
    FK_TRY(need_ws(p));
    if (p->opt.form != FK_FORM_ELL) return fail(FK_ERR_STATE, "plan was not created with FK_FORM_ELL");
    if (n < 0 || n >= p->N) return fail(FK_ERR_ARG, "step outside [0, N-1]");
    if (!cols || !vals || !exit_mass) return fail(FK_ERR_ARG, "null output");
    hipStream_t s = (hipStream_t)stream;
    int *icols = (int *)p->at("ell_org");
    void *ivals = p->at("ell_vals"), *iem = p->at("ell_em");
    FK_LAUNCH(fk::launch_tables(p->dev, n, s));
    FK_LAUNCH(fk::launch_assemble_ell(p->dev, p->f32, n, icols, ivals, iem, s));
    FK_LAUNCH(fk::launch_export_ell(p->dev, p->f32, icols, ivals, cols, vals, s));
    FK_HIP(hipMemcpyAsync(exit_mass, iem, (size_t)p->n_active * elt(p), hipMemcpyDeviceToDevice, s));
    return FK_OK;
}

fk_status fk_check_flags(fk_plan *p, void *stream, int *flags)
{
    FK_TRY(need_ws(p));
    if (!flags) return fail(FK_ERR_ARG, "null flags");
    hipStream_t s = (hipStream_t)stream;
    int h = 0;
    FK_HIP(hipMemcpyAsync(&h, p->at("flags"), sizeof(int), hipMemcpyDeviceToHost, s));
    FK_HIP(hipStreamSynchronize(s));
    FK_LAUNCH(fk::launch_clear_flags(p->dev, s));
    if (p->sub) {
        int hs = 0;
        fk_status st = fk_check_flags(p->sub, stream, &hs);
        if (st != FK_OK && st != FK_ERR_NONFINITE && st != FK_ERR_UNSUPPORTED) return st;
        h |= hs;
    }
    *flags = h;
    if (h & 1) return fail(FK_ERR_NONFINITE, "a non-finite value was produced");
    if (h & 2) return fail(FK_ERR_UNSUPPORTED, "a landing point fell outside the ELL row box");
    return FK_OK;
}

static fk_status prof_mark(fk_plan *p, int kind, hipStream_t s)
{
    if (!p->prof) return FK_OK;
    hipEvent_t e;
    FK_HIP(hipEventCreate(&e));
    FK_HIP(hipEventRecord(e, s));
    p->prof->push_back({e, kind});
    return FK_OK;
}

fk_status fk_adjoint(fk_plan *p, const void *lam0, double *grad, void *lamN, void *stream)
{
    FK_TRY(need_ws(p));
    if (p->opt.ckpt_every <= 0) return fail(FK_ERR_STATE, "plan created without ckpt_every > 0");
    if (!lam0 || !grad) return fail(FK_ERR_ARG, "null lam0 or grad");
    hipStream_t s = (hipStream_t)stream;
    const size_t fb = elt(p) * (size_t)p->n_nodes;
    const int K = p->opt.ckpt_every;
    // 1. forward pass storing checkpoints, unless the latest fk_forward on this
    //    stream stored them already
    if (!(p->ckpt_valid && p->ckpt_stream == s)) {
        p->ckpt_valid = false;
        FK_TRY(enqueue_pass(p, nullptr, p->N, nullptr, 0, nullptr, s, true));
        p->ckpt_valid = true;
        p->ckpt_stream = s;
    }
    // 2. reverse sweep, segment by segment from step 0 upward
    void *la = p->at("lamA"), *lb = p->at("lamB"), *mu = p->at("mu");
    double *g = (double *)p->at("grad");
    unsigned char *ck = (unsigned char *)p->at("ckpt");
    unsigned char *seg = (unsigned char *)p->at("seg");
    void *packed = p->at("packed");
    FK_LAUNCH(fk::launch_zero(g, sizeof(double) * fk::kThetaSlots * p->n_inst, s));
    FK_LAUNCH(fk::launch_adjoint_init(p->dev, p->f32, lam0, la, s, p->conv));
    // the per-step passes touch only the nodes a step can reach and leave mu
    // clear behind them: clear mu and the second lam buffer once
    FK_LAUNCH(fk::launch_zero(mu, fb * rec_stride(p->d), s));
    FK_LAUNCH(fk::launch_zero(lb, fb, s));
    const int nseg = (p->N - 1) / K + 1;
    for (int sg = 0; sg < nseg; ++sg) {
        const int n0 = sg * K, n1 = std::min(n0 + K, p->N);
        const int top_slot = (n1 == p->N) ? p->n_ckpt - 1 : n1 / K;
        // u^{m} for m in (n0, n1]: the top from its checkpoint slot, the rest
        // recomputed into seg[m - n0 - 1]
        const unsigned char *top = ck + (size_t)top_slot * fb;
        auto field = [&](int m) -> const void * {
            return m == n1 ? (const void *)top : (const void *)(seg + (size_t)(m - n0 - 1) * fb);
        };
        for (int m = n1 - 1; m >= n0 + 1; --m) {
            void *dst = seg + (size_t)(m - n0 - 1) * fb;
            FK_LAUNCH(fk::launch_init_field(p->dev, p->f32, dst, s));
            FK_TRY(prof_mark(p, -1, s));
            FK_TRY(enqueue_step(p, m, field(m + 1), dst, s));
            FK_TRY(prof_mark(p, 3, s));
        }
        for (int n = n0; n < n1; ++n) {
            const void *v = field(n + 1);   // u^{n+1}
            FK_TRY(prof_mark(p, -1, s));
            FK_LAUNCH(fk::launch_slopes(p->dev, p->f32, n, v, packed, s));
            FK_TRY(prof_mark(p, 0, s));
            if (p->prof) {
                FK_LAUNCH(fk::launch_adjoint_step(p->dev, p->f32, n, packed, la, mu, g, s, 1));
                FK_TRY(prof_mark(p, 1, s));
                FK_LAUNCH(fk::launch_adjoint_step(p->dev, p->f32, n, packed, la, mu, g, s, 2));
                FK_TRY(prof_mark(p, 4, s));
            } else {
                FK_LAUNCH(fk::launch_adjoint_step(p->dev, p->f32, n, packed, la, mu, g, s));
            }
            FK_LAUNCH(fk::launch_adjoint_slopes_T(p->dev, p->f32, v, mu, lb, s));
            FK_TRY(prof_mark(p, 2, s));
            std::swap(la, lb);
        }
    }
    if (p->conv) {
        // child: gradient rows and dJ/du^N into the parent's outputs
        for (int k = 0; k < p->n_inst; ++k)
            FK_HIP(hipMemcpyAsync(grad + (size_t)p->parent_inst[k] * fk::kThetaSlots,
                                  g + (size_t)k * fk::kThetaSlots, sizeof(double) * fk::kThetaSlots,
                                  hipMemcpyDeviceToDevice, s));
        if (lamN) FK_LAUNCH(fk::launch_convert_out(p->dev, (const double *)la, (float *)lamN, s));
        return FK_OK;
    }
    FK_HIP(hipMemcpyAsync(grad, g, sizeof(double) * fk::kThetaSlots * p->n_inst,
                          hipMemcpyDeviceToDevice, s));
    if (lamN) FK_HIP(hipMemcpyAsync(lamN, la, fb, hipMemcpyDeviceToDevice, s));
    if (p->sub) FK_TRY(fk_adjoint(p->sub, lam0, grad, lamN, stream));
    return FK_OK;
}

fk_status fk_profile_pass(fk_plan *p, double *ms, int *counts, void *stream)
{
    FK_TRY(need_ws(p));
    if (!ms || !counts) return fail(FK_ERR_ARG, "null output");
    hipStream_t s = (hipStream_t)stream;
    const int nk = 4;
    std::vector<hipEvent_t> ev;
    std::vector<int> kind;
    auto rec = [&](int k) -> fk_status {
        hipEvent_t e;
        FK_HIP(hipEventCreate(&e));
        FK_HIP(hipEventRecord(e, s));
        ev.push_back(e);
        kind.push_back(k);
        return FK_OK;
    };
    void *ua = p->at("uA"), *ub = p->at("uB"), *packed = p->at("packed");
    FK_LAUNCH(fk::launch_init_field(p->dev, p->f32, ua, s));
    FK_LAUNCH(fk::launch_init_field(p->dev, p->f32, ub, s));
    void *cur = ua, *nxt = ub;
    for (int n = p->N - 1; n >= 0; --n) {
        FK_TRY(rec(-1));
        FK_LAUNCH(fk::launch_slopes(p->dev, p->f32, n, cur, packed, s));
        FK_TRY(rec(0));
        if (p->opt.form == FK_FORM_ELL) {
            int *cols = (int *)p->at("ell_org");
            void *vals = p->at("ell_vals"), *em = p->at("ell_em");
            FK_LAUNCH(fk::launch_assemble_ell(p->dev, p->f32, n, cols, vals, em, s));
            FK_TRY(rec(2));
            FK_LAUNCH(fk::launch_ell_apply(p->dev, p->f32, cols, vals, em, packed, nxt, s));
            FK_TRY(rec(3));
        } else {
            FK_LAUNCH(fk::launch_step_fused(p->dev, p->f32, n, packed, nxt, s));
            FK_TRY(rec(1));
        }
        std::swap(cur, nxt);
    }
    FK_HIP(hipStreamSynchronize(s));
    double tot[nk] = {0, 0, 0, 0};
    int cnt[nk] = {0, 0, 0, 0};
    for (size_t i = 1; i < ev.size(); ++i) {
        if (kind[i] < 0) continue;
        float t = 0.f;
        FK_HIP(hipEventElapsedTime(&t, ev[i - 1], ev[i]));
        tot[kind[i]] += t;
        cnt[kind[i]] += 1;
    }
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    for (int k = 0; k < nk; ++k) {
        ms[k] = cnt[k] ? tot[k] / cnt[k] : 0.0;
        counts[k] = cnt[k];
    }
    return FK_OK;
}

fk_status fk_tune(const fk_problem *probs, int n_inst, const fk_options *opt, int trial_steps,
                  void *workspace, size_t workspace_bytes, void *stream, fk_tune_result *out)
{
    if (!probs || n_inst < 1 || !out) return fail(FK_ERR_ARG, "null problems or result");
    if (trial_steps < 1) return fail(FK_ERR_ARG, "trial_steps must be >= 1");
    if (!workspace) return fail(FK_ERR_ARG, "null workspace");
    hipStream_t s = (hipStream_t)stream;
    std::vector<fk_problem> trial(probs, probs + n_inst);
    for (fk_problem &pr : trial) pr.n_steps = std::min(pr.n_steps, trial_steps);
    fk_options base{};
    if (opt) base = *opt;
    base.ckpt_every = 0;
    std::memset(out, 0, sizeof(*out));
    double best = 1e300;
    std::vector<std::pair<int, int>> seen;   // (step_kind, use_box) already timed
    for (int sk = 1; sk <= 4; ++sk) {
        fk_options o = base;
        o.step_kernel = sk;
        fk_plan *p = nullptr;
        if (fk_plan_create(trial.data(), n_inst, &o, &p) != FK_OK) {
            g_err.clear();   // layout not compiled for this plan: skip it
            continue;
        }
        const std::pair<int, int> key{p->step_kind, p->use_box ? 1 : 0};
        bool dup = false;
        for (const auto &k : seen) dup = dup || k == key;
        if (dup) {
            fk_plan_destroy(p);
            continue;
        }
        seen.push_back(key);
        if (p->ws_bytes > workspace_bytes) {
            const size_t need = p->ws_bytes;
            fk_plan_destroy(p);
            return fail(FK_ERR_WORKSPACE, "trial plan needs %zu workspace bytes, %zu given", need,
                        workspace_bytes);
        }
        fk_status st = fk_plan_set_workspace(p, workspace, workspace_bytes, stream);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        float ms = 0.f;
        if (st == FK_OK) st = fk_forward(p, nullptr, 0, nullptr, stream);   // warm-up / capture
        if (st == FK_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
            st = fail(FK_ERR_HIP, "event create");
        if (st == FK_OK && hipEventRecord(e0, s) != hipSuccess) st = fail(FK_ERR_HIP, "event record");
        if (st == FK_OK) st = fk_forward(p, nullptr, 0, nullptr, stream);
        if (st == FK_OK && hipEventRecord(e1, s) != hipSuccess) st = fail(FK_ERR_HIP, "event record");
        if (st == FK_OK && hipEventSynchronize(e1) != hipSuccess) st = fail(FK_ERR_HIP, "event sync");
        if (st == FK_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            st = fail(FK_ERR_HIP, "event timing");
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        const int steps = p->N;
        fk_plan_destroy(p);
        if (st != FK_OK) return st;
        out->ms_per_step[sk] = ms / steps;
        if (out->ms_per_step[sk] < best) {
            best = out->ms_per_step[sk];
            out->step_kernel = sk;
        }
    }
    if (out->step_kernel == 0) return fail(FK_ERR_UNSUPPORTED, "no step layout could be built");
    return FK_OK;
}

fk_status fk_probe_lds_atomics(int f32, double *adds_per_s, void *workspace, size_t workspace_bytes,
                               void *stream)
{
    const int blocks = 2048, iters = 4096;
    if (!adds_per_s || !workspace) return fail(FK_ERR_ARG, "null argument");
    if (workspace_bytes < sizeof(double) * blocks)
        return fail(FK_ERR_WORKSPACE, "probe needs %zu bytes", sizeof(double) * blocks);
    hipStream_t s = (hipStream_t)stream;
    double *out = (double *)workspace;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    FK_HIP(hipEventCreate(&e0));
    FK_HIP(hipEventCreate(&e1));
    fk_status st = FK_OK;
    float best = 1e30f;
    for (int rep = 0; rep < 4 && st == FK_OK; ++rep) {
        float ms = 0.f;
        if (hipEventRecord(e0, s) != hipSuccess ||
            fk::launch_lds_atomic_probe(f32 != 0, blocks, iters, out, s) != hipSuccess ||
            hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            st = fail(FK_ERR_HIP, "LDS atomic probe");
        if (rep > 0) best = std::min(best, ms);   // the first run warms up
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st == FK_OK) *adds_per_s = (double)blocks * 256.0 * iters / (best * 1e-3);
    return st;
}

fk_status fk_probe_precision(const fk_problem *probs, int n_inst, const fk_options *opt,
                             double tol, const double *lam0, double grad_tol, void *workspace,
                             size_t workspace_bytes, void *stream, size_t *bytes_needed,
                             int *force_f64, double *diff, double *grad_diff)
{
    if (!probs || n_inst < 1) return fail(FK_ERR_ARG, "null problems");
    if (!(tol > 0)) return fail(FK_ERR_ARG, "tol must be > 0");
    if (lam0 && !(grad_tol > 0)) return fail(FK_ERR_ARG, "grad_tol must be > 0");
    if (!workspace && !bytes_needed) return fail(FK_ERR_ARG, "null workspace and size output");
    if (workspace && (!force_f64 || !diff)) return fail(FK_ERR_ARG, "null outputs");
    hipStream_t s = (hipStream_t)stream;
    std::vector<fk_problem> pr(probs, probs + n_inst);
    for (fk_problem &q : pr) q.force_f64 = 0;
    fk_options o{};
    if (opt) o = *opt;
    o.form = FK_FORM_FUSED;
    o.ckpt_every = lam0 || !workspace ? kProbeCkpt : 0;
    fk_plan *p64 = nullptr, *p32 = nullptr;
    o.precision = FK_PREC_F64;
    FK_TRY(fk_plan_create(pr.data(), n_inst, &o, &p64));
    o.precision = FK_PREC_F32;
    fk_status st = fk_plan_create(pr.data(), n_inst, &o, &p32);
    if (st != FK_OK) {
        fk_plan_destroy(p64);
        return st;
    }
    const size_t nn = (size_t)p64->n_nodes, ni = (size_t)n_inst;
    const size_t o32 = align_up(p64->ws_bytes), of64 = o32 + align_up(p32->ws_bytes);
    const size_t of32 = of64 + align_up(8 * nn), odiff = of32 + align_up(4 * nn);
    const size_t olam = odiff + align_up(8 * ni), og64 = olam + align_up(4 * nn);
    const size_t og32 = og64 + align_up(8 * fk::kThetaSlots * ni);
    const size_t need = og32 + align_up(8 * fk::kThetaSlots * ni);
    if (bytes_needed) *bytes_needed = need;
    if (workspace) {
        unsigned char *ws = (unsigned char *)workspace;
        if (((uintptr_t)ws) % kAlign) st = fail(FK_ERR_ARG, "workspace must be 256-byte aligned");
        else if (workspace_bytes < need)
            st = fail(FK_ERR_WORKSPACE, "probe needs %zu workspace bytes, %zu given", need,
                      workspace_bytes);
        const int snap = 0;
        double *u64 = (double *)(ws + of64);
        float *u32 = (float *)(ws + of32);
        double *dd = (double *)(ws + odiff);
        float *lam32 = (float *)(ws + olam);
        double *g64 = (double *)(ws + og64), *g32 = (double *)(ws + og32);
        if (st == FK_OK) st = fk_plan_set_workspace(p64, ws, p64->ws_bytes, stream);
        if (st == FK_OK) st = fk_plan_set_workspace(p32, ws + o32, p32->ws_bytes, stream);
        if (st == FK_OK) st = fk_forward(p64, &snap, 1, u64, stream);
        if (st == FK_OK) st = fk_forward(p32, &snap, 1, u32, stream);
        if (st == FK_OK && fk::launch_zero(dd, 8 * ni, s) != hipSuccess)
            st = fail(FK_ERR_HIP, "clear");
        if (st == FK_OK && fk::launch_inst_maxdiff(p64->dev, u64, u32, dd, s) != hipSuccess)
            st = fail(FK_ERR_HIP, "difference kernel");
        if (st == FK_OK && hipMemcpyAsync(diff, dd, 8 * ni, hipMemcpyDeviceToHost, s) != hipSuccess)
            st = fail(FK_ERR_HIP, "copy");
        std::vector<double> h64(fk::kThetaSlots * ni), h32(fk::kThetaSlots * ni);
        if (lam0) {
            // the same cotangent, rounded to FP32 for the FP32 plan
            if (st == FK_OK && fk::launch_convert_out(p32->dev, lam0, lam32, s) != hipSuccess)
                st = fail(FK_ERR_HIP, "convert");
            if (st == FK_OK) st = fk_adjoint(p64, lam0, g64, nullptr, stream);
            if (st == FK_OK) st = fk_adjoint(p32, lam32, g32, nullptr, stream);
            if (st == FK_OK && (hipMemcpyAsync(h64.data(), g64, 8 * h64.size(), hipMemcpyDeviceToHost, s) != hipSuccess ||
                                hipMemcpyAsync(h32.data(), g32, 8 * h32.size(), hipMemcpyDeviceToHost, s) != hipSuccess))
                st = fail(FK_ERR_HIP, "copy");
        }
        if (st == FK_OK && hipStreamSynchronize(s) != hipSuccess) st = fail(FK_ERR_HIP, "sync");
        if (st == FK_OK) {
            const int nt = p64->n_theta;
            for (int i = 0; i < n_inst; ++i) {
                bool f = !(diff[i] <= 0.5 * tol);
                double gd = 0.0;
                if (lam0) {
                    double gmax = 0.0, dmax = 0.0;
                    for (int k = 0; k < nt; ++k) {
                        const double a = h64[(size_t)i * fk::kThetaSlots + k];
                        const double b = h32[(size_t)i * fk::kThetaSlots + k];
                        gmax = std::max(gmax, std::fabs(a));
                        dmax = std::max(dmax, std::fabs(a - b));
                        if (!(std::fabs(a - b) >= 0)) dmax = HUGE_VAL;   // NaN
                    }
                    gd = dmax == 0.0 ? 0.0 : (gmax > 0.0 ? dmax / gmax : HUGE_VAL);
                    f = f || !(gd <= 0.5 * grad_tol);
                }
                force_f64[i] = f ? 1 : 0;
                if (grad_diff) grad_diff[i] = gd;
            }
        }
    }
    fk_plan_destroy(p64);
    fk_plan_destroy(p32);
    return st;
}

fk_status fk_profile_adjoint(fk_plan *p, const void *lam0, double *grad, double *ms,
                             int *counts, void *stream)
{
    FK_TRY(need_ws(p));
    if (!ms || !counts) return fail(FK_ERR_ARG, "null output");
    hipStream_t s = (hipStream_t)stream;
    std::vector<std::pair<hipEvent_t, int>> ev;
    p->prof = &ev;
    const fk_status st = fk_adjoint(p, lam0, grad, nullptr, stream);
    p->prof = nullptr;
    fk_status rs = st;
    if (st == FK_OK && hipStreamSynchronize(s) != hipSuccess) rs = fail(FK_ERR_HIP, "stream sync");
    const int nk = 5;
    double tot[nk] = {0, 0, 0, 0, 0};
    int cnt[nk] = {0, 0, 0, 0, 0};
    for (size_t i = 1; rs == FK_OK && i < ev.size(); ++i) {
        if (ev[i].second < 0) continue;
        float t = 0.f;
        if (hipEventElapsedTime(&t, ev[i - 1].first, ev[i].first) != hipSuccess) {
            rs = fail(FK_ERR_HIP, "event timing");
            break;
        }
        tot[ev[i].second] += t;
        cnt[ev[i].second] += 1;
    }
    for (auto &e : ev) (void)hipEventDestroy(e.first);
    for (int k = 0; k < nk; ++k) {
        ms[k] = cnt[k] ? tot[k] / cnt[k] : 0.0;
        counts[k] = cnt[k];
    }
    return rs;
}

}  // extern "C"
