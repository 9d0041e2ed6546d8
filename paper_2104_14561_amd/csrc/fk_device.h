// fk_device.h -- gfx950 device code of the backward Feynman-Kac step.
//
// Kernels are templates here; the launcher sources (fk_launch.hip and the
// per-(precision, dimension) instances of fk_node_inst.hip) instantiate them,
// so that the library builds as several translation units in parallel.
//
// One backward step u^{n+1} -> u^n (paper Section 3.1, Scheme 1; matrix form
// u^n = Q Psi^n F^n u^{n+1}, Eq. (e36)) is two passes:
//   1. slope pass (F^n): per node near the active region, the PCHIP slope
//      along every axis (Eq. (e300) and the end-node rule after it), packed
//      with the value into one record (u, g_0, .., g_{d-1}) so that the step
//      pass gathers a whole cell corner with one vector load.  The same launch
//      tabulates sin/cos of the per-axis arguments of the drift at t_n.
//   2. step pass (Q Psi^n): per active node, the Euler landing points through
//      the tensor Gauss-Hermite nodes (Eq. (e31)), exit test, cell location,
//      tensor cubic Hermite weights (Section 3.1.2) and the weighted sum over
//      quadrature points (Eq. (quad)).
//
// Lane layout of the step pass: a group of G lanes (G = Q rounded up to a
// power of two, at most one wave) serves one active node; lane l takes the
// tensor Gauss-Hermite points q = l, l + G, ...  The sum over the group is a
// fixed shuffle tree, so FP64 results are reproducible run to run.  The sum
// is accumulated as offsets from the node's own value u^{n+1}_j
// (u^n_j = u^{n+1}_j + sum_q w_q (v_q - u^{n+1}_j), v_q = 1 for an exit), which
// is the same number in exact arithmetic (sum_q w_q = 1) but keeps the
// rounding of weights and basis in FP32 proportional to the local variation
// of u instead of u itself.
//
// Landing points, exit tests and cells are FP64 in both precisions; the
// evaluation order of the landing point is sq = sqrt(2 dt), S = sqrt(2D) sq,
// c = x + b dt, z = c + S a, with every product rounded (no contraction), so
// that cells agree bit for bit with any implementation that follows the same
// order.
#pragma once

#include "fk_internal.h"

#include <cmath>

namespace fk {
namespace {

constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// Packed node record (u, slopes): 2 entries for d = 1, 4 for d = 2, 3.
// ---------------------------------------------------------------------------
template <typename T, int PS> struct RecT;
template <> struct RecT<double, 2> { using type = double2; };
template <> struct RecT<double, 4> { using type = double4; };
template <> struct RecT<float, 2> { using type = float2; };
template <> struct RecT<float, 4> { using type = float4; };

template <int D> struct RecStride { static constexpr int value = (D == 1) ? 2 : 4; };

// ---------------------------------------------------------------------------
// Work distribution: a persistent loop over work items.  Workgroups are
// dispatched round-robin over the 8 XCDs (workgroup b runs on XCD b % 8);
// each XCD takes a contiguous chunk of the work list so that neighbouring
// tiles -- whose stencils overlap -- share one L2.
// ---------------------------------------------------------------------------
struct WorkRange {
    int begin, end, step;
};

__device__ inline WorkRange work_range(int first, int n_work)
{
    const int nx = 8;
    const int g = gridDim.x;
    WorkRange r;
    if (g < nx || (g % nx) != 0) {
        r.begin = first + blockIdx.x;
        r.end = first + n_work;
        r.step = g;
        return r;
    }
    const int xcd = blockIdx.x % nx, local = blockIdx.x / nx, per = g / nx;
    const int chunk = (n_work + nx - 1) / nx;
    r.begin = first + xcd * chunk + local;
    r.end = first + min(n_work, (xcd + 1) * chunk);
    r.step = per;
    return r;
}

// ---------------------------------------------------------------------------
// Axis geometry.  An affine axis (host-verified: x_k = k * step + lo exactly
// for k < n-1, x_{n-1} = hi) needs no coordinate loads.
// ---------------------------------------------------------------------------
__device__ inline double coord(const DevInst &I, const double *coords, int a, int k)
{
#pragma clang fp contract(off)
    if (I.affine[a]) return (k == I.n[a] - 1) ? I.hi[a] : (double)k * I.step[a] + I.lo[a];
    return coords[I.coord_off[a] + k];
}

// Cell of z: max{k : x_k <= z}, clamped to [0, n-2].  On a uniform axis the
// arithmetic guess floor((z - lo) / h) is within one cell of the answer (the
// spacing deviates from h by far less than a cell), so one conditional step up
// and one down against the node coordinates give it exactly; other axes use
// binary search over the stored coordinates.
__device__ inline int locate(const DevInst &I, const double *coords, int a, double z)
{
    const int n = I.n[a];
    int k;
    if (I.uniform[a]) {
        const double f = floor((z - I.lo[a]) * I.inv_h[a]);
        k = (f >= 0.0) ? ((f <= (double)(n - 2)) ? (int)f : n - 2) : 0;
        if (k < n - 2 && coord(I, coords, a, k + 1) <= z) ++k;
        if (k > 0 && coord(I, coords, a, k) > z) --k;
    } else {
        const double *x = coords + I.coord_off[a];
        int l = 0, h = n - 1;
        if (z >= x[n - 1]) {
            l = n - 2;
        } else if (z >= x[0]) {
            while (h - l > 1) {
                const int m = (l + h) >> 1;
                if (x[m] <= z) l = m; else h = m;
            }
        }
        k = l;
    }
    return k;
}

// One axis of a landing point: coordinate, exit flag, cell and position.
struct AxisEval {
    double s;      // position inside the cell
    double h;      // cell width
    double dz2;    // (z - centre)^2 for the ball test
    int k;         // cell
    bool ex;       // z left the box on this (non-periodic) axis
    double exv;    // the value it takes then (1, or 0 through an exit-0 face)
};

__device__ inline AxisEval eval_axis(const DevInst &I, const double *coords, int a, double c,
                                     double ga)
{
#pragma clang fp contract(off)
    double z = c + I.S * ga;
    if (I.periodic[a]) {
        if (z >= I.hi[a]) z = z - I.period[a];
        else if (z < I.lo[a]) z = z + I.period[a];
    }
    AxisEval e;
    e.ex = !I.periodic[a] && (z <= I.lo[a] || z >= I.hi[a]);
    const double t = z - I.center[a];
    e.dz2 = t * t;
    const int k = locate(I, coords, a, z);
    const double xk = coord(I, coords, a, k);
    if (I.affine[a]) {
        e.h = I.step[a];
        e.s = (z - xk) * I.inv_h[a];
    } else {
        e.h = coord(I, coords, a, k + 1) - xk;
        e.s = (z - xk) / e.h;
    }
    e.k = k;
    return e;
}

// Axis evaluation for an affine axis (x_k = k * step + lo exactly, x_{n-1} =
// hi): the floor guess and the exact one-step fix-ups without loads or loops.
__device__ inline AxisEval eval_axis_affine(const DevInst &I, int a, double c, double ga)
{
#pragma clang fp contract(off)
    double z = c + I.S * ga;
    const double lo = I.lo[a], hi = I.hi[a];
    if (I.periodic[a]) {
        if (z >= hi) z = z - I.period[a];
        else if (z < lo) z = z + I.period[a];
    }
    AxisEval e;
    e.ex = !I.periodic[a] && (z <= lo || z >= hi);
    const double t = z - I.center[a];
    e.dz2 = t * t;
    const int n = I.n[a];
    const double step = I.step[a];
    const double f = floor((z - lo) * I.inv_h[a]);
    int k = (f >= 0.0) ? ((f <= (double)(n - 2)) ? (int)f : n - 2) : 0;
    const double xk1 = (k + 1 == n - 1) ? hi : (double)(k + 1) * step + lo;
    if (k < n - 2 && xk1 <= z) ++k;
    double xk = (double)k * step + lo;
    if (k > 0 && xk > z) {
        --k;
        xk = (double)k * step + lo;
    }
    e.k = k;
    e.h = step;
    e.s = (z - xk) * I.inv_h[a];
    return e;
}

// Axis evaluation with the node's own scale S (S = sigma_a sqrt(2 dt)) and
// the instance's face kinds: a reflecting face mirrors z back into the
// domain (z -> lo + (lo - z)); an exit face records the value it gives.
__device__ inline AxisEval eval_axis_faces(const DevInst &I, const double *coords, int a,
                                           double c, double ga, double S)
{
#pragma clang fp contract(off)
    double z = c + S * ga;
    const double lo = I.lo[a], hi = I.hi[a];
    AxisEval e;
    e.ex = false;
    e.exv = 1.0;
    if (I.periodic[a]) {
        if (z >= hi) z = z - I.period[a];
        else if (z < lo) z = z + I.period[a];
    } else {
        const int fl = I.face[a][0], fh = I.face[a][1];
        if (fl == 2 && z < lo) z = lo + (lo - z);
        if (fh == 2 && z > hi) z = hi - (z - hi);
        if (fl != 2 && z <= lo) {
            e.ex = true;
            e.exv = fl == 1 ? 0.0 : 1.0;
        } else if (fh != 2 && z >= hi) {
            e.ex = true;
            e.exv = fh == 1 ? 0.0 : 1.0;
        }
    }
    const double t = z - I.center[a];
    e.dz2 = t * t;
    const int k = locate(I, coords, a, z);
    const double xk = coord(I, coords, a, k);
    if (I.affine[a]) {
        e.h = I.step[a];
        e.s = (z - xk) * I.inv_h[a];
    } else {
        e.h = coord(I, coords, a, k + 1) - xk;
        e.s = (z - xk) / e.h;
    }
    e.k = k;
    return e;
}

template <bool AFF>
__device__ inline AxisEval eval_axis_t(const DevInst &I, const double *coords, int a, double c,
                                       double ga)
{
    if constexpr (AFF) return eval_axis_affine(I, a, c, ga);
    else return eval_axis(I, coords, a, c, ga);
}

__device__ inline bool ball_exit2(double a, double b, double r2)
{
#pragma clang fp contract(off)
    double s = a;
    s = s + b;
    return s >= r2;
}

__device__ inline bool ball_exit(const double *dz2, int d, double r2)
{
#pragma clang fp contract(off)
    double s = dz2[0];
    for (int a = 1; a < d; ++a) s = s + dz2[a];
    return s >= r2;
}

// ---------------------------------------------------------------------------
// Coefficients (FP64).  tf = per-(step, instance) time factors tabulated at
// plan creation: cellular (eps sin(omega t), sin(omega t), cos(omega t), t);
// ABC (1 + amp sin t, sin t, 0, t).  trig = per-axis (sin, cos) table of the
// drift's argument at each node coordinate for the current step:
// cellular axis 0: pi (x + eps sin(omega t)); cellular axis 1: pi y;
// ABC: the coordinate itself; rolls (Section 4.2 example): axis 0 n x,
// axis 1 pi y (the roll count n is coef[3]).
// ---------------------------------------------------------------------------
__device__ inline double trig_arg(const DevInst &I, const double *tf, int a, double x)
{
#pragma clang fp contract(off)
    if (I.coef_kind == 1) return (a == 0) ? M_PI * (x + tf[0]) : M_PI * x;
    if (I.coef_kind == 3) return (a == 0) ? I.coef[3] * x : M_PI * x;
    return x;
}

template <int D>
__device__ inline void drift(const DevInst &I, const double *tf, const double2 *trig,
                             const int *idx, double *b)
{
#pragma clang fp contract(off)
    if (I.coef_kind == 0) {
#pragma unroll
        for (int a = 0; a < D; ++a) b[a] = I.coef[a];
    } else if (I.coef_kind == 1) {
        const double2 t0 = trig[I.coord_off[0] + idx[0]];
        const double2 t1 = trig[I.coord_off[1] + idx[1]];
        const double sa = t0.x, ca = t0.y, sy = t1.x, cy = t1.y;
        const double Api = I.coef[0] * M_PI;
        b[0] = -(Api * sa * cy);
        b[1] = Api * ca * sy;
    } else if (I.coef_kind == 3) {
        // rolls: Pe v with v_1 = -pi cos(pi y) (sin(n x) + e cos(n x)),
        // v_2 = n sin(pi y) (cos(n x) - e sin(n x)), e = eps cos(omega t)
        const double2 t0 = trig[I.coord_off[0] + idx[0]];
        const double2 t1 = trig[I.coord_off[1] + idx[1]];
        const double s1 = t0.x, c1 = t0.y, s2 = t1.x, c2 = t1.y;
        const double e = tf[0];
        b[0] = -(I.coef[0] * M_PI * c2 * (s1 + e * c1));
        b[1] = I.coef[0] * I.coef[3] * s2 * (c1 - e * s1);
    } else {
        const double2 tx = trig[I.coord_off[0] + idx[0]];
        const double2 ty = trig[I.coord_off[1] + idx[1]];
        const double2 tz = trig[I.coord_off[2] + idx[2]];
        const double f = tf[0];
        const double Af = I.coef[0] * f, Bf = I.coef[1] * f, Cf = I.coef[2] * f;
        b[0] = Af * tz.x + Cf * ty.y;
        b[1] = Bf * tx.x + Af * tz.y;
        b[2] = Cf * ty.x + Bf * tx.y;
    }
}

// d b_a / d theta_k for the drift parameters (theta_k, k < np); db[k*3 + a].
template <int D>
__device__ inline int drift_dtheta(const DevInst &I, const double *tf, const double2 *trig,
                                   const int *idx, double *db)
{
#pragma unroll
    for (int k = 0; k < 12; ++k) db[k] = 0.0;
    if (I.coef_kind == 0) {
#pragma unroll
        for (int a = 0; a < D; ++a) db[a * 3 + a] = 1.0;
        return D;
    } else if (I.coef_kind == 1) {
        const double A = I.coef[0], eps = I.coef[1];
        const double swt = tf[1], cwt = tf[2], t = tf[3];
        const double2 t0 = trig[I.coord_off[0] + idx[0]];
        const double2 t1 = trig[I.coord_off[1] + idx[1]];
        const double sphi = t0.x, cphi = t0.y, sy = t1.x, cy = t1.y;
        const double db0 = -A * M_PI * cphi * cy;   // d b0 / d phi
        const double db1 = -A * M_PI * sphi * sy;   // d b1 / d phi
        const double dpe = M_PI * swt;              // d phi / d eps
        const double dpo = M_PI * eps * t * cwt;    // d phi / d omega
        db[0] = -M_PI * sphi * cy;  db[1] = M_PI * cphi * sy;
        db[3] = db0 * dpe;          db[4] = db1 * dpe;
        db[6] = db0 * dpo;          db[7] = db1 * dpo;
        return 3;
    } else if (I.coef_kind == 3) {
        // rolls: theta = (Pe, eps, omega); e = eps cos(omega t)
        const double Pe = I.coef[0], eps = I.coef[1], nn = I.coef[3];
        const double e = tf[0], cwt = tf[1], swt = tf[2], t = tf[3];
        const double2 t0 = trig[I.coord_off[0] + idx[0]];
        const double2 t1 = trig[I.coord_off[1] + idx[1]];
        const double s1 = t0.x, c1 = t0.y, s2 = t1.x, c2 = t1.y;
        const double db0 = -(Pe * M_PI * c2 * c1);   // d b0 / d e
        const double db1 = -(Pe * nn * s2 * s1);     // d b1 / d e
        const double dee = cwt;                      // d e / d eps
        const double deo = -(eps * t * swt);         // d e / d omega
        db[0] = -(M_PI * c2 * (s1 + e * c1));  db[1] = nn * s2 * (c1 - e * s1);
        db[3] = db0 * dee;                     db[4] = db1 * dee;
        db[6] = db0 * deo;                     db[7] = db1 * deo;
        return 3;
    } else {
        const double A = I.coef[0], B = I.coef[1], C = I.coef[2];
        const double f = tf[0], st = tf[1];
        const double2 tx = trig[I.coord_off[0] + idx[0]];
        const double2 ty = trig[I.coord_off[1] + idx[1]];
        const double2 tz = trig[I.coord_off[2] + idx[2]];
        const double sx = tx.x, cx = tx.y, sy = ty.x, cy = ty.y, sz = tz.x, cz = tz.y;
        db[0] = f * sz;  db[1] = f * cz;                      // A
        db[4] = f * sx;  db[5] = f * cx;                      // B
        db[6] = f * cy;  db[8] = f * sy;                      // C
        db[9] = st * (A * sz + C * cy);                        // amp
        db[10] = st * (B * sx + A * cz);
        db[11] = st * (C * sy + B * cx);
        return 4;
    }
}

template <int D>
__device__ inline void split_node(const DevInst &I, int node, int *idx)
{
    if (D == 1) {
        idx[0] = node;
    } else if (D == 2) {
        idx[0] = node / I.n[1];
        idx[1] = node - idx[0] * I.n[1];
    } else {
        const int plane = I.n[1] * I.n[2];
        idx[0] = node / plane;
        const int rem = node - idx[0] * plane;
        idx[1] = rem / I.n[2];
        idx[2] = rem - idx[1] * I.n[2];
    }
}

// Landing-point centre c = x + b(t_n, x) dt of a node.
template <int D>
__device__ inline void node_centre(const DevInst &I, const double *coords, const double *tf,
                                   const double2 *trig, const int *idx, double dt, double *c)
{
#pragma clang fp contract(off)
    double b[3];
    drift<D>(I, tf, trig, idx, b);
    for (int a = 0; a < D; ++a) c[a] = coord(I, coords, a, idx[a]) + b[a] * dt;
}

// Runaway-electron model (Section 4.3, Eq. (ex32d)) at node idx: the
// landing-point centre c = x + b dt and the per-axis scales S_a = sigma_a
// sqrt(2 dt), with the collision functions of phi = erf, psi = (phi - y phi')
// / (2 y^2), y = p / gamma, and the radial tanh transition.  tf = (E, nu_ee,
// v_T, delta) at t_n (tabulated on the host).  Operation order as written
// (no contraction).
__device__ inline void runaway_centre(const DevInst &I, const double *coords, const double *tf,
                                      const int *idx, double dt, double *c, double *S)
{
#pragma clang fp contract(off)
    const double *p = I.coef;
    const double E = tf[0], nu = tf[1], vT = tf[2], delta = tf[3];
    const double pm = coord(I, coords, 0, idx[0]);
    const double xi = coord(I, coords, 1, idx[1]);
    const double r = coord(I, coords, 2, idx[2]);
    const double gam = sqrt(1.0 + (delta * pm) * (delta * pm));
    const double om = 1.0 - xi * xi;
    const double y = pm / gam;
    const double phi = erf(y);
    const double dphi = 2.0 / sqrt(M_PI) * exp(-y * y);
    const double psi = (phi - y * dphi) / (2.0 * y * y);
    const double dpsi = dphi - 2.0 * psi / y;
    const double k2 = nu * vT * vT;
    const double CA = k2 * psi / y;
    const double CB = 0.5 * k2 / y * (p[2] + phi - psi + 0.5 * y * y * pow(delta, 4.0));
    const double CF = 2.0 * nu * vT * psi;
    const double dCA = k2 * (dpsi * y - psi) / (y * y) / (gam * gam * gam);
    const double th = tanh((r - p[6]) / p[7]);
    const double ep = exp(-(pm / p[8]) * (pm / p[8]));
    const double Dr = 0.5 * p[10] * (1.0 + th) * ep;
    const double dDr = 0.5 * p[10] * (1.0 - th * th) / p[7] * ep;
    double b[3];
    b[0] = E * xi - gam * pm / p[1] * om - CF + 2.0 * CA / pm + dCA;
    b[1] = E * om / pm - xi * om / (p[1] * gam) - 2.0 * xi * CB / (pm * pm);
    b[2] = (r > p[6] ? p[9] : 0.0) + dDr;
    const double x[3] = {pm, xi, r};
    for (int a = 0; a < 3; ++a) c[a] = x[a] + b[a] * dt;
    const double sq = sqrt(2.0 * dt);
    S[0] = sqrt(2.0 * CA) * sq;
    S[1] = sqrt(2.0 * CB) / pm * sqrt(om > 0.0 ? om : 0.0) * sq;
    S[2] = sqrt(2.0 * Dr) * sq;
}

// Centre and per-axis scales of any model (S_a = the instance's S unless the
// diffusion depends on the node).
template <int D>
__device__ inline void node_centre_s(const DevInst &I, const double *coords, const double *tf,
                                     const double2 *trig, const int *idx, double dt, double *c,
                                     double *S)
{
    if constexpr (D == 3) {
        if (I.sdiff) {
            runaway_centre(I, coords, tf, idx, dt, c, S);
            return;
        }
    }
    node_centre<D>(I, coords, tf, trig, idx, dt, c);
    for (int a = 0; a < D; ++a) S[a] = I.S;
}

// ---------------------------------------------------------------------------
// Cubic Hermite basis on [0, 1] (Section 3.1.2): value basis v0 = H00,
// v1 = H01 and slope basis times the cell width d0 = h H10, d1 = h H11, and
// the derivatives of both with respect to z.
// ---------------------------------------------------------------------------
template <typename T> struct Basis {
    T v0, v1, d0, d1;
};

template <typename T>
__device__ inline Basis<T> hermite(double s_d, double h_d)
{
    const T s = (T)s_d, h = (T)h_d;
    const T om = T(1) - s;
    Basis<T> B;
    B.v0 = (T(1) + T(2) * s) * om * om;
    B.v1 = s * s * (T(3) - T(2) * s);
    B.d0 = h * s * om * om;
    B.d1 = h * s * s * (s - T(1));
    return B;
}

template <typename T>
__device__ inline Basis<T> hermite_dz(double s_d, double h_d)
{
    const T s = (T)s_d, h = (T)h_d;
    Basis<T> B;
    B.v0 = (T(6) * s * s - T(6) * s) / h;
    B.v1 = (T(6) * s - T(6) * s * s) / h;
    B.d0 = T(1) - T(4) * s + T(3) * s * s;
    B.d1 = T(3) * s * s - T(2) * s;
    return B;
}

template <int G, typename T>
__device__ inline T group_sum(T v)
{
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename T>
__device__ inline void flag_nonfinite(int *flags, T v)
{
    if (!isfinite((double)v)) atomicOr(flags, 1);
}

// Write a node's value and its periodic images.
template <int D, typename T>
__device__ inline void store_node(const DevInst &I, const int *idx, long long node, T v,
                                  T *u_out)
{
    u_out[I.node_off + node] = v;
    int pm = 0;
    for (int a = 0; a < D; ++a)
        if (I.periodic[a] && idx[a] == 0) pm |= 1 << a;
    if (pm) {
        for (int sub = pm; sub; sub = (sub - 1) & pm) {
            long long o = node;
            for (int a = 0; a < D; ++a)
                if (sub & (1 << a)) o += (long long)(I.n[a] - 1) * I.stride[a];
            u_out[I.node_off + o] = v;
        }
    }
}

// Hermite value of the corner records p at one landing point; the value
// entries enter as offsets (p.x - uref).  TW (2D): the R2 interpolant, whose
// records carry the twist field in their fourth entry.
template <typename T, int D, typename R, bool TW = false>
__device__ inline T hermite_value(const R *p, const Basis<T> *B, T uref)
{
    if constexpr (D == 1) {
        return (p[0].x - uref) * B[0].v0 + (p[1].x - uref) * B[0].v1 + p[0].y * B[0].d0 +
               p[1].y * B[0].d1;
    } else if constexpr (D == 2) {
        // corners p[a*2 + b]: a along axis 0, b along axis 1
        const Basis<T> &X = B[0], &Y = B[1];
        const T A0 = (p[0].x - uref) * X.v0 + (p[2].x - uref) * X.v1 + p[0].y * X.d0 + p[2].y * X.d1;
        const T A1 = (p[1].x - uref) * X.v0 + (p[3].x - uref) * X.v1 + p[1].y * X.d0 + p[3].y * X.d1;
        T C0 = p[0].z * X.v0 + p[2].z * X.v1;
        T C1 = p[1].z * X.v0 + p[3].z * X.v1;
        if constexpr (TW) {
            C0 += p[0].w * X.d0 + p[2].w * X.d1;
            C1 += p[1].w * X.d0 + p[3].w * X.d1;
        }
        return Y.v0 * A0 + Y.v1 * A1 + Y.d0 * C0 + Y.d1 * C1;
    } else {
        // corners p[(a*2 + b)*2 + c]
        const Basis<T> &X = B[0], &Y = B[1], &Z = B[2];
        T acc = T(0);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const T Zv = c ? Z.v1 : Z.v0, Zd = c ? Z.d1 : Z.d0;
            T sv = T(0), sd = T(0);
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const T Yv = b ? Y.v1 : Y.v0, Yd = b ? Y.d1 : Y.d0;
                const R &p0 = p[(0 * 2 + b) * 2 + c], &p1 = p[(1 * 2 + b) * 2 + c];
                const T xu = (p0.x - uref) * X.v0 + (p1.x - uref) * X.v1 + p0.y * X.d0 + p1.y * X.d1;
                const T xg1 = p0.z * X.v0 + p1.z * X.v1;
                const T xg2 = p0.w * X.v0 + p1.w * X.v1;
                sv += Yv * xu + Yd * xg1;
                sd += Yv * xg2;
            }
            acc += Zv * sv + Zd * sd;
        }
        return acc;
    }
}

// The R2 interpolant in 3D: corner records p (u, g0, g1, g2) and q (t01, t02,
// t12, t012), corners [(a*2 + b)*2 + c]; the field of axis set S weighted by
// the slope bases of S and the value bases of the other axes.
template <typename T, typename R>
__device__ inline T hermite_value3_tw(const R *p, const R *q, const Basis<T> *B, T uref)
{
    const Basis<T> &X = B[0], &Y = B[1], &Z = B[2];
    T acc = T(0);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const T Zv = c ? Z.v1 : Z.v0, Zd = c ? Z.d1 : Z.d0;
        T sv = T(0), sd = T(0);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const T Yv = b ? Y.v1 : Y.v0, Yd = b ? Y.d1 : Y.d0;
            const int k0 = (0 * 2 + b) * 2 + c, k1 = (1 * 2 + b) * 2 + c;
            const R &p0 = p[k0], &p1 = p[k1], &q0 = q[k0], &q1 = q[k1];
            // fields with S restricted to axis 0 given the (axis 1, axis 2) part
            const T x00 = (p0.x - uref) * X.v0 + (p1.x - uref) * X.v1 + p0.y * X.d0 + p1.y * X.d1;
            const T x10 = p0.z * X.v0 + p1.z * X.v1 + q0.x * X.d0 + q1.x * X.d1;   // g1, t01
            const T x01 = p0.w * X.v0 + p1.w * X.v1 + q0.y * X.d0 + q1.y * X.d1;   // g2, t02
            const T x11 = q0.z * X.v0 + q1.z * X.v1 + q0.w * X.d0 + q1.w * X.d1;   // t12, t012
            sv += Yv * x00 + Yd * x10;
            sd += Yv * x01 + Yd * x11;
        }
        acc += Zv * sv + Zd * sd;
    }
    return acc;
}

// Gradient of the Hermite value with respect to z (adjoint); Bz = hermite_dz.
template <typename T, int D, typename R>
__device__ inline void hermite_grad(const R *p, const Basis<T> *B, const Basis<T> *Bz, T *g)
{
    Basis<T> BB[3];
    for (int m = 0; m < D; ++m) {
        for (int a = 0; a < D; ++a) BB[a] = (a == m) ? Bz[a] : B[a];
        g[m] = hermite_value<T, D, R>(p, BB, T(0));
    }
}

// Gather the 2^D corner records of a cell.
template <int D, typename R>
__device__ inline void gather_corners(const R *rec, const DevInst &I, const int *k, R *p)
{
    long long base = I.node_off;
    for (int a = 0; a < D; ++a) base += (long long)k[a] * I.stride[a];
    if constexpr (D == 1) {
        p[0] = rec[base];
        p[1] = rec[base + 1];
    } else if constexpr (D == 2) {
        const long long s0 = I.stride[0];
        p[0] = rec[base];
        p[1] = rec[base + 1];
        p[2] = rec[base + s0];
        p[3] = rec[base + s0 + 1];
    } else {
        const long long s0 = I.stride[0], s1 = I.stride[1];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                p[(a * 2 + b) * 2 + 0] = rec[base + a * s0 + b * s1];
                p[(a * 2 + b) * 2 + 1] = rec[base + a * s0 + b * s1 + 1];
            }
    }
}

// Landing point with the GH coordinates aq[] of the point already known.
template <int D>
__device__ inline bool landing_point_a(const DevInst &I, const double *coords, const double *c,
                                       const double *aq, int *k, double *s, double *h)
{
    bool ex = false;
    double dz2[3];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const AxisEval e = eval_axis(I, coords, a, c[a], aq[a]);
        ex = ex || e.ex;
        dz2[a] = e.dz2;
        k[a] = e.k;
        s[a] = e.s;
        h[a] = e.h;
    }
    if (I.region_kind == 1) ex = ex || ball_exit(dz2, D, I.r2);
    return ex;
}

// Evaluates landing point q of a node: exit flag, cells and per-axis data.
template <int D>
__device__ inline bool landing_point(const DevInst &I, const double *coords, const double *ga,
                                     int qs, const double *c, int q, int *k, double *s, double *h)
{
    double aq[3];
    for (int a = D - 1; a >= 0; --a) {
        aq[a] = ga[q % qs];
        q /= qs;
    }
    bool ex = false;
    double dz2[3];
    for (int a = 0; a < D; ++a) {
        const AxisEval e = eval_axis(I, coords, a, c[a], aq[a]);
        ex = ex || e.ex;
        dz2[a] = e.dz2;
        k[a] = e.k;
        s[a] = e.s;
        h[a] = e.h;
    }
    if (I.region_kind == 1) ex = ex || ball_exit(dz2, D, I.r2);
    return ex;
}

template <typename T> __device__ inline const T *weights(const PlanDev &P);
template <> __device__ inline const double *weights<double>(const PlanDev &P) { return P.gh_w; }
template <> __device__ inline const float *weights<float>(const PlanDev &P) { return P.gh_wf; }

template <typename T> __device__ inline const T *weights1(const PlanDev &P);
template <> __device__ inline const double *weights1<double>(const PlanDev &P) { return P.gh_w1; }
template <> __device__ inline const float *weights1<float>(const PlanDev &P) { return P.gh_w1f; }

__device__ inline const double *time_factors(const PlanDev &P, int n, int inst)
{
    return P.tfac + ((long long)n * P.n_inst + inst) * kTimeFactors;
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

template <typename T>
__global__ void __launch_bounds__(kBlock) k_init_field(const unsigned char *cls, long long n,
                                                       T *u)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        u[i] = (T)((cls[i] & 5) == 1 ? 1 : 0);   // bit 2: an exit node of value 0
}

// Stencil of the PCHIP slope along axis a at index i (Eq. (e300) and the end
// rule after it): the three nodes along the axis and the two spacings.
__device__ inline void slope_stencil(const DevInst &I, const double *coords, int a, int i,
                                     int &il, int &ic, int &ir, double &hl, double &hr)
{
    const int na = I.n[a];
    if (I.periodic[a]) {
        ic = (i == na - 1) ? 0 : i;
        il = (ic == 0) ? na - 2 : ic - 1;
        ir = ic + 1;
    } else if (i == 0) {
        il = 0; ic = 1; ir = 2;
    } else if (i == na - 1) {
        il = na - 3; ic = na - 2; ir = na - 1;
    } else {
        il = i - 1; ic = i; ir = i + 1;
    }
    if (I.affine[a]) {
        hl = I.step[a];
        hr = I.step[a];
    } else {
        const double *x = coords + I.coord_off[a];
        hl = (ic == 0) ? x[na - 1] - x[na - 2] : x[ic] - x[il];
        hr = x[ir] - x[ic];
    }
}

template <typename T>
__device__ inline T pchip_slope(T dl, T dr)
{
    return (dl * dr > T(0)) ? T(2) * dl * dr / (dl + dr) : T(0);
}

// Twist field of the R2 interpolant at node idx of a 2D instance: the PCHIP
// slope along axis 1 of the axis-0 slopes at the three nodes of its axis-1
// stencil (each from the axis-0 stencil of that row).
template <typename T>
__device__ inline T twist_2d(const DevInst &I, const double *coords, const T *ui, const int *idx)
{
    int il0, ic0, ir0, il1, ic1, ir1;
    double hl0, hr0, hl1, hr1;
    slope_stencil(I, coords, 0, idx[0], il0, ic0, ir0, hl0, hr0);
    slope_stencil(I, coords, 1, idx[1], il1, ic1, ir1, hl1, hr1);
    const long long s0 = I.stride[0];
    auto g0 = [&](int j) -> T {
        const T ul = ui[il0 * s0 + j], uc = ui[ic0 * s0 + j], ur = ui[ir0 * s0 + j];
        return pchip_slope<T>((uc - ul) / (T)hl0, (ur - uc) / (T)hr0);
    };
    const T gl = g0(il1), gc = g0(ic1), gr = g0(ir1);
    return pchip_slope<T>((gc - gl) / (T)hl1, (gr - gc) / (T)hr1);
}

// R2 twist fields in 3D at node idx: t01 = D_1(D_0 u), t02 = D_2(D_0 u),
// t12 = D_2(D_1 u), t012 = D_2(t01) -- each the PCHIP slope along the largest
// axis of its set of the field of the set without that axis, the lower fields
// recomputed at the stencil nodes with the same rule.
template <typename T>
__device__ inline void twist_3d(const DevInst &I, const double *coords, const T *ui, const int *idx,
                                T *tw)
{
    int l[3][3];
    double hl[3], hr[3];
    for (int a = 0; a < 3; ++a) slope_stencil(I, coords, a, idx[a], l[a][0], l[a][1], l[a][2], hl[a], hr[a]);
    const long long s0 = I.stride[0], s1 = I.stride[1];
    auto at = [&](int i0, int i1, int i2) -> T { return ui[i0 * s0 + i1 * s1 + i2]; };
    // slope along axis 0 at (i0 = idx0's stencil, i1, i2)
    auto g0 = [&](int i1, int i2) -> T {
        const T ul = at(l[0][0], i1, i2), uc = at(l[0][1], i1, i2), ur = at(l[0][2], i1, i2);
        return pchip_slope<T>((uc - ul) / (T)hl[0], (ur - uc) / (T)hr[0]);
    };
    auto g1 = [&](int i2) -> T {
        const T ul = at(idx[0], l[1][0], i2), uc = at(idx[0], l[1][1], i2), ur = at(idx[0], l[1][2], i2);
        return pchip_slope<T>((uc - ul) / (T)hl[1], (ur - uc) / (T)hr[1]);
    };
    auto t01 = [&](int i2) -> T {
        const T gl = g0(l[1][0], i2), gc = g0(l[1][1], i2), gr = g0(l[1][2], i2);
        return pchip_slope<T>((gc - gl) / (T)hl[1], (gr - gc) / (T)hr[1]);
    };
    auto along2 = [&](T fl, T fc, T fr) -> T {
        return pchip_slope<T>((fc - fl) / (T)hl[2], (fr - fc) / (T)hr[2]);
    };
    tw[0] = t01(idx[2]);
    tw[1] = along2(g0(idx[1], l[2][0]), g0(idx[1], l[2][1]), g0(idx[1], l[2][2]));
    tw[2] = along2(g1(l[2][0]), g1(l[2][1]), g1(l[2][2]));
    tw[3] = along2(t01(l[2][0]), t01(l[2][1]), t01(l[2][2]));
}

// Slope pass for step n over work items [first, first + count): table items
// (kind 1 + a) fill the (sin, cos) table of axis a; node items (kind 0) write
// record[node] = (u, g_0, .., g_{d-1}).
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_slopes(PlanDev P, int n, int first, int count,
                                                   const T *__restrict__ u,
                                                   T *__restrict__ packed)
{
    constexpr int PS = RecStride<D>::value;
    using R = typename RecT<T, PS>::type;
    R *rec = reinterpret_cast<R *>(packed);
    const WorkRange wr = work_range(first, count);
    for (int w = wr.begin; w < wr.end; w += wr.step) {
        const WorkItem it = P.slope_work[w];
        if ((int)threadIdx.x >= it.count) continue;
        const DevInst &I = P.inst[it.inst];
        if (it.kind > 0) {
            const int a = it.kind - 1;
            const int i = it.first + threadIdx.x;
            const double arg = trig_arg(I, time_factors(P, n, it.inst), a,
                                        P.coords[I.coord_off[a] + i]);
            P.trig[I.coord_off[a] + i] = make_double2(sin(arg), cos(arg));
            continue;
        }
        const int node = it.first + threadIdx.x;
        int idx[3];
        split_node<D>(I, node, idx);
        const T *ui = u + I.node_off;
        T out[4] = {ui[node], T(0), T(0), T(0)};
        for (int a = 0; a < D; ++a) {
            const int na = I.n[a];
            const int i = idx[a];
            int il, ic, ir;
            if (I.periodic[a]) {
                ic = (i == na - 1) ? 0 : i;
                il = (ic == 0) ? na - 2 : ic - 1;
                ir = ic + 1;
            } else if (i == 0) {
                il = 0; ic = 1; ir = 2;
            } else if (i == na - 1) {
                il = na - 3; ic = na - 2; ir = na - 1;
            } else {
                il = i - 1; ic = i; ir = i + 1;
            }
            double hl, hr;
            if (I.affine[a]) {
                hl = I.step[a];
                hr = I.step[a];
            } else {
                const double *x = P.coords + I.coord_off[a];
                hl = (ic == 0) ? x[na - 1] - x[na - 2] : x[ic] - x[il];
                hr = x[ir] - x[ic];
            }
            const long long base = node - (long long)i * I.stride[a];
            const T ul = ui[base + (long long)il * I.stride[a]];
            const T uc = ui[base + (long long)ic * I.stride[a]];
            const T ur = ui[base + (long long)ir * I.stride[a]];
            const T dl = (uc - ul) / (T)hl;
            const T dr = (ur - uc) / (T)hr;
            out[1 + a] = (dl * dr > T(0)) ? T(2) * dl * dr / (dl + dr) : T(0);
        }
        if constexpr (D == 2) {
            // R2 twist: the PCHIP slope along axis 1 of the axis-0 slope field
            // (the one-dimensional rule composed in increasing axis order)
            if (P.hermite2) out[3] = twist_2d<T>(I, P.coords, ui, idx);
        } else if constexpr (D == 3) {
            // R2: the four twist fields in the node's second record
            if (P.hermite2) {
                T tw[4];
                twist_3d<T>(I, P.coords, ui, idx, tw);
                R q;
                q.x = tw[0]; q.y = tw[1]; q.z = tw[2]; q.w = tw[3];
                reinterpret_cast<R *>(P.packed2)[I.node_off + node] = q;
            }
        }
        R r;
        if constexpr (PS == 2) {
            r.x = out[0]; r.y = out[1];
        } else {
            r.x = out[0]; r.y = out[1]; r.z = out[2]; r.w = out[3];
        }
        rec[I.node_off + node] = r;
    }
}

// Per-axis data of one landing coordinate, shared through LDS by the lanes of
// a node's group.  The tensor rule makes every per-axis quantity depend only on
// (axis, 1D Gauss-Hermite index), so a node needs d Q* of these, not d Q.
template <typename T> struct AxisRec {
    int k;        // cell
    int ex;       // left the box on this axis: 0 no, 1 with value 1, 2 with value 0
    double dz2;   // (z - centre)^2
    T v0, v1, d0, d1;
};

// Fills the node's axis records: lane l < d Q* evaluates axis l / Q* at GH
// index l % Q*.
template <typename T, int D>
__device__ inline void stage_axes(const DevInst &I, const double *coords, const double *gh_a,
                                  int qs, const double *c, int lane, AxisRec<T> *tab,
                                  const double *S, bool faces)
{
    if (lane < D * qs) {
        const int a = lane / qs, qa = lane - a * qs;
        const double ca = (D == 1 || a == 0) ? c[0] : (a == 1 ? c[1] : c[2]);
        const double Sa = (D == 1 || a == 0) ? S[0] : (a == 1 ? S[1] : S[2]);
        const AxisEval e = faces ? eval_axis_faces(I, coords, a, ca, gh_a[qa], Sa)
                                 : eval_axis(I, coords, a, ca, gh_a[qa]);
        const Basis<T> B = hermite<T>(e.s, e.h);
        AxisRec<T> r;
        r.k = e.k;
        r.ex = e.ex ? (e.exv == 0.0 ? 2 : 1) : 0;
        r.dz2 = e.dz2;
        r.v0 = B.v0; r.v1 = B.v1; r.d0 = B.d0; r.d1 = B.d1;
        tab[lane] = r;
    }
}

// Fused step pass (matrix-free form of Eq. (e36)).  A group of G lanes serves
// one active node: its d Q* axis evaluations are staged in LDS, then lane l
// assembles the tensor points q = l, l + G, ... (at most NQ), gathers the cell
// corners' records and contracts them with the tensor Hermite weights.  The
// read-only tables come in as restrict-qualified arguments so that
// per-instance fields are fetched with scalar loads.
template <typename T, int D, int G, int NQ>
__global__ void __launch_bounds__(kBlock) k_step_fused(
    const PlanDev P, int n, const DevInst *__restrict__ insts,
    const WorkItem *__restrict__ work, const int *__restrict__ active,
    const double2 *__restrict__ trig, const double *__restrict__ coords,
    const T *__restrict__ packed, T *__restrict__ u_out)
{
    constexpr int PS = RecStride<D>::value;
    using R = typename RecT<T, PS>::type;
    constexpr int NPB = kBlock / G;
    __shared__ AxisRec<T> tabs[NPB][G];
    const R *rec = reinterpret_cast<const R *>(packed);
    const int lane = threadIdx.x % G;
    int slot = threadIdx.x / G;
    if (G == 64) slot = __builtin_amdgcn_readfirstlane(slot);
    AxisRec<T> *tab = tabs[slot];
    const int qs = P.qs;
    // this lane's tensor points q = lane + i G: per-axis GH indices and weight
    int qa[NQ][3];
    T wq[NQ];
    bool has[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        int q = lane + i * G;
        has[i] = q < P.n_quad;
        if (!has[i]) q = 0;
        wq[i] = has[i] ? weights<T>(P)[q] : T(0);
        for (int a = D - 1; a >= 0; --a) {
            qa[i][a] = a * qs + q % qs;
            q /= qs;
        }
    }
    const WorkRange wr = work_range(0, P.n_act_work);
    for (int w = wr.begin; w < wr.end; w += wr.step) {
        const WorkItem it = work[w];
        const bool valid = slot < it.count;
        const DevInst &I = insts[it.inst];
        T acc = T(0), uref = T(0);
        int idx[3] = {0, 0, 0};
        int node = 0;
        if (valid) {
            node = active[I.act_off + it.first + slot];
            split_node<D>(I, node, idx);
            uref = rec[I.node_off + node].x;
            double c[3], S[3];
            node_centre_s<D>(I, coords, time_factors(P, n, it.inst), trig, idx, P.dt, c, S);
            stage_axes<T, D>(I, coords, P.gh_a, qs, c, lane, tab, S, P.faces != 0);
        }
        __syncthreads();
        if (valid) {
            const bool ball = I.region_kind == 1;
#pragma unroll
            for (int i = 0; i < NQ; ++i) {
                if (!has[i]) continue;
                AxisRec<T> ar[3];
                bool ex = false;
                T xv = T(1);   // value of an exit: the lowest exiting axis decides
                double dz2[3];
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    ar[a] = tab[qa[i][a]];
                    if (!ex && ar[a].ex == 2) xv = T(0);
                    ex = ex || ar[a].ex;
                    dz2[a] = ar[a].dz2;
                }
                if (ball) ex = ex || ball_exit(dz2, D, I.r2);
                if (ex) {
                    acc += wq[i] * (xv - uref);
                } else {
                    Basis<T> B[3];
                    int k[3];
#pragma unroll
                    for (int a = 0; a < D; ++a) {
                        k[a] = ar[a].k;
                        B[a].v0 = ar[a].v0; B[a].v1 = ar[a].v1;
                        B[a].d0 = ar[a].d0; B[a].d1 = ar[a].d1;
                    }
                    R p[1 << D];
                    gather_corners<D, R>(rec, I, k, p);
                    if (D == 2 && P.hermite2)
                        acc += wq[i] * hermite_value<T, D, R, true>(p, B, uref);
                    else
                        acc += wq[i] * hermite_value<T, D, R>(p, B, uref);
                }
            }
        }
        acc = group_sum<G>(acc);
        if (valid && lane == 0) {
            const T v = uref + acc;
            flag_nonfinite(P.flags, v);
            store_node<D, T>(I, idx, node, v, u_out);
        }
        __syncthreads();
    }
}

// Thread-per-node fused step (the main path).  Lane = active node; the
// innermost axis' QS landing coordinates (cell, Hermite basis, exit flag and
// ball distance) are evaluated once per node and kept in registers, the outer
// axes are looped.  Consecutive lanes are consecutive nodes along the fastest
// axis, so one gather instruction of a wave reads neighbouring records.  The
// exit mass is summed over exiting points only (zero when none exits), so the
// rounding of FP32 weights never biases nodes far from the exit region.
//
// G > 1 (small plans): G lanes share a node, lane l taking the outermost
// axis' indices l, l + G, ...; the lane sums are combined by a shuffle tree.
//
// FC: face kinds other than exit-1 and node-dependent diffusion (the
// runaway model): the node's own per-axis scales, reflecting faces mirrored
// by the axis evaluation, and a second exit mass for exits with value 0 (the
// lowest exiting axis decides a point's value, as in the loops' order).  In
// FP32 up to Q* = 4 it is held to 3 waves per SIMD (167 VGPRs, a few spilled;
// measured on the runaway model at Q* = 4: 124 against 140 us per step at the
// 2 waves of its 183 VGPRs).
template <typename T, int D, int QS, int G, bool AFF, bool TW = false, bool FC = false>
__global__ void __launch_bounds__(kBlock, (FC && sizeof(T) == 4 && QS <= 4) ? 3 : 1) k_step_node(
    const PlanDev P, int n, int n_work, const DevInst *__restrict__ insts,
    const WorkItem *__restrict__ work, const int *__restrict__ nodes,
    const double2 *__restrict__ trig, const double *__restrict__ coords,
    const T *__restrict__ packed, T *__restrict__ u_out)
{
    constexpr int PS = RecStride<D>::value;
    using R = typename RecT<T, PS>::type;
    const R *rec = reinterpret_cast<const R *>(packed);
    const double *ga = P.gh_a;
    const T *w1 = weights1<T>(P);
    T wsum = T(0);
#pragma unroll
    for (int q = 0; q < QS; ++q) wsum += w1[q];
    const int lane = (G > 1) ? (int)(threadIdx.x % G) : 0;
    const int slot = (G > 1) ? (int)(threadIdx.x / G) : (int)threadIdx.x;
    const WorkRange wr = work_range(0, n_work);
    for (int w = wr.begin; w < wr.end; w += wr.step) {
        const WorkItem it = work[w];
        if (G == 1 && slot >= it.count) continue;
        const bool valid = slot < it.count;
        const bool interior = !FC && it.kind == 1;   // host: no landing point can exit
        const DevInst &I = insts[it.inst];
        const int node = valid ? nodes[it.first + slot] : nodes[it.first];
        int idx[3];
        split_node<D>(I, node, idx);
        const T uref = rec[I.node_off + node].x;
        double c[3], S[3] = {0.0, 0.0, 0.0};
        if constexpr (FC) node_centre_s<D>(I, coords, time_factors(P, n, it.inst), trig, idx, P.dt, c, S);
        else node_centre<D>(I, coords, time_factors(P, n, it.inst), trig, idx, P.dt, c);
        // one landing coordinate on axis a
        auto axis = [&](int a, double g) -> AxisEval {
            if constexpr (FC) return eval_axis_faces(I, coords, a, c[a], g, S[a]);
            else return eval_axis_t<AFF>(I, coords, a, c[a], g);
        };
        const bool ball = I.region_kind == 1;
        const double r2 = I.r2;
        // innermost axis, hoisted
        constexpr int AI = D - 1;
        int kin[QS];
        T bin[QS][4];
        bool exin[QS], ex0in[QS];
        double din[QS];
#pragma unroll
        for (int q = 0; q < QS; ++q) {
            const AxisEval e = axis(AI, ga[q]);
            const Basis<T> B = hermite<T>(e.s, e.h);
            kin[q] = e.k;
            bin[q][0] = B.v0; bin[q][1] = B.v1; bin[q][2] = B.d0; bin[q][3] = B.d1;
            exin[q] = e.ex;
            ex0in[q] = FC && e.ex && e.exv == 0.0;
            din[q] = e.dz2;
        }
        // exit masses: value 1 (emass) and, with FC, value 0 (em0)
        T acc = T(0), emass = T(0), em0 = T(0);
        if constexpr (D == 1) {
#pragma unroll
            for (int q = 0; q < QS; ++q) {
                if (G > 1 && (q % G) != lane) continue;
                const bool ex = exin[q] || (ball && din[q] >= r2);
                if (ex) {
                    if (ex0in[q]) em0 += w1[q];
                    else emass += w1[q];
                    continue;
                }
                const long long base = I.node_off + kin[q];
                const R p0 = rec[base], p1 = rec[base + 1];
                const T v = (p0.x - uref) * bin[q][0] + (p1.x - uref) * bin[q][1] +
                            p0.y * bin[q][2] + p1.y * bin[q][3];
                acc += w1[q] * v;
            }
        } else if constexpr (D == 2) {
            // records of the instance, indexed with 32-bit offsets
            const R *ri = rec + I.node_off;
            const int s0 = I.stride[0];
            // landing point (q0, q1) of a cell row: the tensor Hermite value
            auto point = [&](int row, const Basis<T> &X, int q1) -> T {
                const int b = row + kin[q1];
                const R p00 = ri[b], p01 = ri[b + 1], p10 = ri[b + s0], p11 = ri[b + s0 + 1];
                const T A0 = (p00.x - uref) * X.v0 + (p10.x - uref) * X.v1 + p00.y * X.d0 + p10.y * X.d1;
                const T A1 = (p01.x - uref) * X.v0 + (p11.x - uref) * X.v1 + p01.y * X.d0 + p11.y * X.d1;
                T C0 = p00.z * X.v0 + p10.z * X.v1;
                T C1 = p01.z * X.v0 + p11.z * X.v1;
                if constexpr (TW) {
                    // R2: the twist field times the slope bases of both axes
                    C0 += p00.w * X.d0 + p10.w * X.d1;
                    C1 += p01.w * X.d0 + p11.w * X.d1;
                }
                return w1[q1] * (bin[q1][0] * A0 + bin[q1][1] * A1 + bin[q1][2] * C0 + bin[q1][3] * C1);
            };
            if (interior) {
                // no landing point of this work item can exit: no exit tests
                for (int q0 = lane; q0 < QS; q0 += G) {
                    const AxisEval e0 = eval_axis_t<AFF>(I, coords, 0, c[0], ga[q0]);
                    const Basis<T> X = hermite<T>(e0.s, e0.h);
                    const int row = e0.k * s0;
                    T part = T(0);
#pragma unroll
                    for (int q1 = 0; q1 < QS; ++q1) part += point(row, X, q1);
                    acc += w1[q0] * part;
                }
            } else {
                for (int q0 = lane; q0 < QS; q0 += G) {
                    const AxisEval e0 = axis(0, ga[q0]);
                    const T w0 = w1[q0];
                    if (e0.ex) {
                        if (FC && e0.exv == 0.0) em0 += w0 * wsum;
                        else emass += w0 * wsum;
                        continue;
                    }
                    const Basis<T> X = hermite<T>(e0.s, e0.h);
                    const int row = e0.k * s0;
                    T part = T(0), pex = T(0), pex0 = T(0);
#pragma unroll
                    for (int q1 = 0; q1 < QS; ++q1) {
                        bool ex = exin[q1];
                        if (ball) ex = ex || ball_exit2(e0.dz2, din[q1], r2);
                        if (ex) {
                            if (ex0in[q1]) pex0 += w1[q1];
                            else pex += w1[q1];
                            continue;
                        }
                        part += point(row, X, q1);
                    }
                    acc += w0 * part;
                    emass += w0 * pex;
                    if constexpr (FC) em0 += w0 * pex0;
                }
            }
        } else {
            for (int q0 = lane; q0 < QS; q0 += G) {
                const AxisEval e0 = axis(0, ga[q0]);
                const T w0 = w1[q0];
                if (e0.ex) {
                    if (FC && e0.exv == 0.0) em0 += w0 * wsum * wsum;
                    else emass += w0 * wsum * wsum;
                    continue;
                }
                const Basis<T> X = hermite<T>(e0.s, e0.h);
                for (int q1 = 0; q1 < QS; ++q1) {
                    const AxisEval e1 = axis(1, ga[q1]);
                    const T w01 = w0 * w1[q1];
                    if (e1.ex) {
                        if (FC && e1.exv == 0.0) em0 += w01 * wsum;
                        else emass += w01 * wsum;
                        continue;
                    }
                    const Basis<T> Y = hermite<T>(e1.s, e1.h);
                    const long long base = I.node_off + (long long)e0.k * I.stride[0] +
                                           (long long)e1.k * I.stride[1];
                    const long long s0 = I.stride[0], s1 = I.stride[1];
                    T part = T(0), pex = T(0), pex0 = T(0);
#pragma unroll
                    for (int q2 = 0; q2 < QS; ++q2) {
                        bool ex = exin[q2];
                        if (ball) {
                            const double dz[3] = {e0.dz2, e1.dz2, din[q2]};
                            ex = ex || ball_exit(dz, 3, r2);
                        }
                        if (ex) {
                            if (ex0in[q2]) pex0 += w1[q2];
                            else pex += w1[q2];
                            continue;
                        }
                        const long long b = base + kin[q2];
                        R p[8];
#pragma unroll
                        for (int a = 0; a < 2; ++a)
#pragma unroll
                            for (int bb = 0; bb < 2; ++bb) {
                                p[(a * 2 + bb) * 2 + 0] = rec[b + a * s0 + bb * s1];
                                p[(a * 2 + bb) * 2 + 1] = rec[b + a * s0 + bb * s1 + 1];
                            }
                        const Basis<T> Z = {bin[q2][0], bin[q2][1], bin[q2][2], bin[q2][3]};
                        const Basis<T> B[3] = {X, Y, Z};
                        if constexpr (TW) {
                            // R2: the corners' twist records
                            const R *rec2 = reinterpret_cast<const R *>(P.packed2);
                            R qq[8];
#pragma unroll
                            for (int a = 0; a < 2; ++a)
#pragma unroll
                                for (int bb = 0; bb < 2; ++bb) {
                                    qq[(a * 2 + bb) * 2 + 0] = rec2[b + a * s0 + bb * s1];
                                    qq[(a * 2 + bb) * 2 + 1] = rec2[b + a * s0 + bb * s1 + 1];
                                }
                            part += w1[q2] * hermite_value3_tw<T, R>(p, qq, B, uref);
                        } else {
                            part += w1[q2] * hermite_value<T, 3, R>(p, B, uref);
                        }
                    }
                    acc += w01 * part;
                    emass += w01 * pex;
                    if constexpr (FC) em0 += w01 * pex0;
                }
            }
        }
        if (G > 1) {
            acc = group_sum<G>(acc);
            emass = group_sum<G>(emass);
            if constexpr (FC) em0 = group_sum<G>(em0);
            if (!valid || lane != 0) continue;
        }
        T v = uref + acc + emass * (T(1) - uref);
        if constexpr (FC) v = v - em0 * uref;
        flag_nonfinite(P.flags, v);
        store_node<D, T>(I, idx, node, v, u_out);
    }
}

// ---------------------------------------------------------------------------
// Separable (box) form.  For a node none of whose landing points can reach a
// ball boundary, the exit test is a per-axis box test and the tensor rule
// factorises: the row of A_n over the footprint box B = B_0 x .. x B_{d-1}
// is sum_a-products of per-axis weight vectors
//   V_a[l] = sum_{q inside on axis a} w_q (H00(s_q) [l = k_q - o_a] + H01(s_q) [l = k_q - o_a + 1])
//   S_a[l] = same with the slope basis h H10, h H11,
// so u^n_j = u_ref + sum_B prod V (u - u_ref) + (slope terms) + exit mass (1 - u_ref),
// exit mass = (sum_q w_q)^d - prod_a m_a, m_a = sum of inside weights on axis a.
// o_a is the (unwrapped) cell of the smallest landing coordinate, and every
// landing cell lies in [o_a, o_a + L - 2] (host bound).
// ---------------------------------------------------------------------------
struct AxisBox {
    int o;       // unwrapped cell of the first GH point
    int n;       // nodes on the axis
    int per;     // periodic
};

// Cell of a landing coordinate, unwrapped across a periodic seam.
template <bool AFF>
__device__ inline AxisEval eval_axis_unwrapped(const DevInst &I, const double *coords, int a,
                                               double c, double ga, int &ku)
{
#pragma clang fp contract(off)
    const AxisEval e = eval_axis_t<AFF>(I, coords, a, c, ga);
    ku = e.k;
    if (I.periodic[a]) {
        const double z = c + I.S * ga;
        if (z >= I.hi[a]) ku += I.n[a] - 1;
        else if (z < I.lo[a]) ku -= I.n[a] - 1;
    }
    return e;
}

// Per-axis weight vectors of one node; returns false if a landing cell left
// the box (cannot happen when the host bound holds).
template <typename T, int QS, int L, bool AFF, bool DERIV>
__device__ inline bool axis_vectors(const DevInst &I, const double *coords, const double *ga,
                                    const T *w1, int a, double c, int &o, T &m, T *V, T *Sv,
                                    T *dV, T *dS, T *aV, T *aS)
{
    bool ok = true;
    m = T(0);
#pragma unroll
    for (int j = 0; j < L; ++j) {
        V[j] = T(0); Sv[j] = T(0);
        if (DERIV) { dV[j] = T(0); dS[j] = T(0); aV[j] = T(0); aS[j] = T(0); }
    }
#pragma unroll
    for (int q = 0; q < QS; ++q) {
        int ku;
        const AxisEval e = eval_axis_unwrapped<AFF>(I, coords, a, c, ga[q], ku);
        if (q == 0) o = ku;
        const int l = ku - o;
        if (l < 0 || l > L - 2) { ok = false; continue; }
        if (e.ex) continue;
        const T w = w1[q];
        m += w;
        const Basis<T> B = hermite<T>(e.s, e.h);
        Basis<T> Bz;
        if (DERIV) Bz = hermite_dz<T>(e.s, e.h);
#pragma unroll
        for (int j = 0; j < L; ++j) {
            const bool a0 = (j == l), a1 = (j == l + 1);
            V[j] += a0 ? w * B.v0 : (a1 ? w * B.v1 : T(0));
            Sv[j] += a0 ? w * B.d0 : (a1 ? w * B.d1 : T(0));
            if (DERIV) {
                const T wa = w * (T)ga[q];
                dV[j] += a0 ? w * Bz.v0 : (a1 ? w * Bz.v1 : T(0));
                dS[j] += a0 ? w * Bz.d0 : (a1 ? w * Bz.d1 : T(0));
                aV[j] += a0 ? wa * Bz.v0 : (a1 ? wa * Bz.v1 : T(0));
                aS[j] += a0 ? wa * Bz.d0 : (a1 ? wa * Bz.d1 : T(0));
            }
        }
    }
    return ok;
}

// Node index of footprint position i on an axis: wrapped across the seam of a
// periodic axis, clamped to the axis otherwise.  Footprint positions past the
// last node carry zero weight (no landing cell reaches them); clamping keeps
// their record reads inside the field.
__device__ inline int wrap_index(int i, int n, int per)
{
    if (per) {
        if (i < 0) i += n - 1;
        else if (i > n - 1) i -= n - 1;
    } else {
        i = i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
    }
    return i;
}

// Box contraction: value and slope-weighted sum over the footprint box of
// the records, with per-axis vector sets (Va, Sa) for each axis.
template <typename T, int D, int L, typename R>
__device__ inline T box_contract(const R *rec, const DevInst &I, const int *o, T uref,
                                 const T (*V)[L], const T (*Sv)[L], bool tw = false)
{
    if constexpr (D == 1) {
        T acc = T(0);
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const R r = rec[I.node_off + wrap_index(o[0] + i, I.n[0], I.periodic[0])];
            acc += V[0][i] * (r.x - uref) + Sv[0][i] * r.y;
        }
        return acc;
    } else if constexpr (D == 2) {
        int j1[L];
#pragma unroll
        for (int j = 0; j < L; ++j) j1[j] = wrap_index(o[1] + j, I.n[1], I.periodic[1]);
        T acc = T(0);
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const long long row = I.node_off +
                (long long)wrap_index(o[0] + i, I.n[0], I.periodic[0]) * I.stride[0];
            T tv = T(0), tg = T(0);
#pragma unroll
            for (int j = 0; j < L; ++j) {
                const R r = rec[row + j1[j]];
                tv += V[1][j] * (r.x - uref) + Sv[1][j] * r.z;
                tg += V[1][j] * r.y;
                if (tw) tg += Sv[1][j] * r.w;   // R2 twist
            }
            acc += V[0][i] * tv + Sv[0][i] * tg;
        }
        return acc;
    } else {
        int j2[L], j1[L];
#pragma unroll
        for (int j = 0; j < L; ++j) {
            j2[j] = wrap_index(o[2] + j, I.n[2], I.periodic[2]);
            j1[j] = wrap_index(o[1] + j, I.n[1], I.periodic[1]);
        }
        T acc = T(0);
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const long long b0 = I.node_off +
                (long long)wrap_index(o[0] + i, I.n[0], I.periodic[0]) * I.stride[0];
            T sv = T(0), sg0 = T(0);
#pragma unroll
            for (int j = 0; j < L; ++j) {
                const long long b1 = b0 + (long long)j1[j] * I.stride[1];
                T tv = T(0), tg0 = T(0), tg1 = T(0);
#pragma unroll
                for (int kk = 0; kk < L; ++kk) {
                    const R r = rec[b1 + j2[kk]];
                    tv += V[2][kk] * (r.x - uref) + Sv[2][kk] * r.w;
                    tg0 += V[2][kk] * r.y;
                    tg1 += V[2][kk] * r.z;
                }
                sv += V[1][j] * tv + Sv[1][j] * tg1;
                sg0 += V[1][j] * tg0;
            }
            acc += V[0][i] * sv + Sv[0][i] * sg0;
        }
        return acc;
    }
}

template <typename T, int D, int QS, int L, bool AFF>
__global__ void __launch_bounds__(kBlock) k_step_box(
    const PlanDev P, int n, int n_work, const DevInst *__restrict__ insts,
    const WorkItem *__restrict__ work, const int *__restrict__ nodes,
    const double2 *__restrict__ trig, const double *__restrict__ coords,
    const T *__restrict__ packed, T *__restrict__ u_out)
{
    constexpr int PS = RecStride<D>::value;
    using R = typename RecT<T, PS>::type;
    const R *rec = reinterpret_cast<const R *>(packed);
    const double *ga = P.gh_a;
    const T *w1 = weights1<T>(P);
    T wsum = T(0);
#pragma unroll
    for (int q = 0; q < QS; ++q) wsum += w1[q];
    const WorkRange wr = work_range(0, n_work);
    for (int w = wr.begin; w < wr.end; w += wr.step) {
        const WorkItem it = work[w];
        if ((int)threadIdx.x >= it.count) continue;
        const DevInst &I = insts[it.inst];
        const int node = nodes[it.first + threadIdx.x];
        int idx[3];
        split_node<D>(I, node, idx);
        const T uref = rec[I.node_off + node].x;
        double c[3];
        node_centre<D>(I, coords, time_factors(P, n, it.inst), trig, idx, P.dt, c);
        T V[D][L], Sv[D][L];
        int o[3];
        T m[3];
        bool ok = true;
#pragma unroll
        for (int a = 0; a < D; ++a)
            ok = axis_vectors<T, QS, L, AFF, false>(I, coords, ga, w1, a, c[a], o[a], m[a], V[a],
                                                    Sv[a], nullptr, nullptr, nullptr, nullptr) && ok;
        if (!ok) atomicOr(P.flags, 2);
        T prod = m[0], wd = wsum;
#pragma unroll
        for (int a = 1; a < D; ++a) { prod *= m[a]; wd *= wsum; }
        const T emass = wd - prod;
        const T acc = box_contract<T, D, L, R>(rec, I, o, uref, V, Sv, P.hermite2 != 0);
        const T v = uref + acc + emass * (T(1) - uref);
        flag_nonfinite(P.flags, v);
        store_node<D, T>(I, idx, node, v, u_out);
    }
}

// Landing cells and exit flags of one instance (index parity checks).
template <int D>
__global__ void __launch_bounds__(kBlock) k_export_cells(PlanDev P, int inst, int n,
                                                         int *cells, unsigned char *exitf)
{
    const DevInst &I = P.inst[inst];
    const long long total = (long long)I.n_act * P.n_quad;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
         t += (long long)gridDim.x * blockDim.x) {
        const int r = (int)(t / P.n_quad);
        const int q = (int)(t - (long long)r * P.n_quad);
        const int node = P.active[I.act_off + r];
        int idx[3];
        split_node<D>(I, node, idx);
        double c[3], S[3];
        node_centre_s<D>(I, P.coords, time_factors(P, n, inst), P.trig, idx, P.dt, c, S);
        int k[3];
        double s[3], h[3];
        bool ex;
        if (P.faces) {
            int qq = q;
            ex = false;
            double dz2[3];
            for (int a = D - 1; a >= 0; --a) {
                const AxisEval e = eval_axis_faces(I, P.coords, a, c[a], P.gh_a[qq % P.qs], S[a]);
                qq /= P.qs;
                ex = ex || e.ex;
                dz2[a] = e.dz2;
                k[a] = e.k;
            }
            if (I.region_kind == 1) ex = ex || ball_exit(dz2, D, I.r2);
        } else {
            ex = landing_point<D>(I, P.coords, P.gh_a, P.qs, c, q, k, s, h);
        }
        exitf[t] = ex ? 1 : 0;
        for (int a = 0; a < D; ++a) cells[t * D + a] = ex ? -1 : k[a];
    }
}

// Add to an LDS entry (workgroup-scope atomic; a different scope from the
// global atomics, so that the compiler keeps the two apart).  The tiles hold
// FP64 in both precisions: on gfx950 an LDS FP64 atomic add issues about ten
// times faster than an FP32 one (measured ~20 against ~200 CU cycles per wave
// instruction), and the tile sum gains precision on the way.
__device__ inline void lds_add(double *p, double v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// ---------------------------------------------------------------------------
// Assembled form (the paper's GPU formulation, Section 3.2.1): A_n stored as
// one dense box per row -- the L_0 x .. x L_{d-1} nodes its landing cells can
// cover (origin: the cell of the smallest landing coordinate on each axis)
// times (d+1) fields -- stored column-major within an instance (entry k of
// all rows, then entry k+1), with the box origin per row.  The columns are
// implicit in the box, so the product streams values only.  The lane group of
// a row builds the box in LDS (FP64 adds); the workgroup writes its rows'
// boxes together, entry by entry.  The stored row is the plain operator
// (u^n_j = exit_mass + A_j [u; g]); the product evaluates it in the same offset
// form as the fused pass.
// ---------------------------------------------------------------------------
// 16 bytes of consecutive box nodes of one field of one row
template <typename T>
struct alignas(16) EllBlock {
    static constexpr int K = 16 / sizeof(T);
    T v[K];
};

// Store a block past the caches' allocation (the values are read back by the
// product only after the whole operator, gigabytes, has been written).
template <typename T>
__device__ inline void store_block_nt(EllBlock<T> *dst, const EllBlock<T> &b)
{
    using V = T __attribute__((ext_vector_type(EllBlock<T>::K)));
    V x;
#pragma unroll
    for (int j = 0; j < EllBlock<T>::K; ++j) x[j] = b.v[j];
    __builtin_nontemporal_store(x, reinterpret_cast<V *>(dst));
}

template <typename T, int D, int G>
__global__ void __launch_bounds__(kBlock) k_assemble_ell(PlanDev P, int n,
                                                         const WorkItem *__restrict__ work,
                                                         int n_work, int bstride,
                                                         int *__restrict__ org,
                                                         T *__restrict__ vals,
                                                         T *__restrict__ exit_mass)
{
    constexpr int PS = RecStride<D>::value;
    extern __shared__ unsigned char smem_raw[];
    double *box = reinterpret_cast<double *>(smem_raw);   // FP64 LDS atomics (fast on gfx950)
    const T *Wq = weights<T>(P);
    const int lane = threadIdx.x % G;
    const int slot = threadIdx.x / G;
    const WorkRange wr = work_range(0, n_work);
    for (int w = wr.begin; w < wr.end; w += wr.step) {
        const WorkItem it = work[w];
        const bool valid = slot < it.count;
        const DevInst &I = P.inst[it.inst];
        const int W = I.ell_w;   // <= bstride, the launch's row-box stride
        double *mybox = box + (long long)slot * bstride;
        for (int k = lane; k < W; k += G) mybox[k] = 0.0;
        __syncthreads();
        int idx[3] = {0, 0, 0};
        int origin[3] = {0, 0, 0};
        T em = T(0);
        long long row = 0;
        if (valid) {
            const int node = P.active[I.act_off + it.first + slot];
            row = I.act_off + it.first + slot;
            split_node<D>(I, node, idx);
            double c[3];
            node_centre<D>(I, P.coords, time_factors(P, n, it.inst), P.trig, idx, P.dt, c);
            // box origin: cell of the smallest landing coordinate per axis
            for (int a = 0; a < D; ++a)
                origin[a] = eval_axis(I, P.coords, a, c[a], P.gh_a[0]).k;
            for (int q = lane; q < P.n_quad; q += G) {
                int k[3];
                double s[3], h[3];
                const bool ex = landing_point<D>(I, P.coords, P.gh_a, P.qs, c, q, k, s, h);
                const T wq = Wq[q];
                if (ex) {
                    em += wq;
                    continue;
                }
                Basis<T> B[3];
                for (int a = 0; a < D; ++a) B[a] = hermite<T>(s[a], h[a]);
                for (int cb = 0; cb < (1 << D); ++cb) {
                    int off = 0;
                    bool in = true;
                    T wv = wq;
                    for (int a = 0; a < D; ++a) {
                        const int bit = (cb >> (D - 1 - a)) & 1;
                        const int l = k[a] + bit - origin[a];
                        in = in && l >= 0 && l < I.ell_box[a];
                        off = off * I.ell_box[a] + l;
                        wv *= bit ? B[a].v1 : B[a].v0;
                    }
                    if (!in) {
                        atomicOr(P.flags, 2);
                        continue;
                    }
                    lds_add(&mybox[off * (D + 1)], (double)wv);
                    for (int a = 0; a < D; ++a) {
                        T ws = wq;
                        for (int i = 0; i < D; ++i) {
                            const int bit = (cb >> (D - 1 - i)) & 1;
                            if (i == a) ws *= bit ? B[i].d1 : B[i].d0;
                            else ws *= bit ? B[i].v1 : B[i].v0;
                        }
                        lds_add(&mybox[off * (D + 1) + 1 + a], (double)ws);
                    }
                }
            }
        }
        em = group_sum<G>(em);
        __syncthreads();
        if (valid && lane == 0) {
            for (int a = 0; a < 3; ++a) org[row * 3 + a] = a < D ? origin[a] : 0;
            exit_mass[row] = em;
        }
        // the workgroup's rows are consecutive: write block b of all of them
        // together.  Block b = f * (nbp / K) + l / K holds value f of box nodes
        // l .. l + K - 1 and sits at (b * rows + r) * K within the instance
        // (blocks of one index are contiguous across rows); padding nodes
        // (l >= nbox) hold 0
        {
            constexpr int K = EllBlock<T>::K;
            const int nrow = it.count;
            const int nbox = W / (D + 1);
            const int bpf = I.ell_nbp / K;   // blocks per field
            const long long rows = I.n_act;
            const long long r0 = it.first;
            // a thread keeps one (row, entry-in-block) pair and walks the blocks
            // with a fixed stride (no division per entry); G >= 4 lanes per row
            // bound nrow by blockDim / 4, so per <= blockDim and nb >= 1
            const int per = nrow * K;                    // entries of one block index
            const int nb = (int)blockDim.x / per;        // block indices per sweep
            const int t = threadIdx.x;
            if (nrow > 0 && t < nb * per) {
                const int rr = (t % per) / K, j = t % K;
                const int nblk = (D + 1) * bpf;
                int b = t / per;
                int f = b / bpf, lb = b - f * bpf;
                T *dst = vals + I.ell_off + (r0 + rr) * K + j;
                const double *src = box + (long long)rr * bstride + f;
                for (; b < nblk; b += nb) {
                    const int l = lb * K + j;
                    dst[(long long)b * rows * K] = l < nbox ? (T)src[l * (D + 1)] : T(0);
                    lb += nb;
                    while (lb >= bpf) {
                        lb -= bpf;
                        ++f;
                        ++src;
                    }
                }
            }
        }
        __syncthreads();
    }
}

// floor(n / d) for 0 <= n, d < 2^16 as a multiply-high: m = floor(2^32 / d) + 1
// makes (n m) >> 32 exact while n d < 2^32.
__device__ inline unsigned long long fast_recip(int d)
{
    return (1ull << 32) / (unsigned long long)d + 1ull;
}
__device__ inline int fast_div(int n, unsigned long long m)
{
    return (int)(((unsigned long long)(unsigned)n * m) >> 32);
}

// Assembly of separable rows (no landing point can reach a curved exit
// boundary; exits through the faces of a box region decide per axis): the
// row is the outer product of per-axis vectors, the value and slope bases of
// that axis summed with its 1D weights over the GH nodes that stay inside, so
// it is written directly, with no LDS atomics.  A workgroup takes up to 64
// rows (a lane per row); wave a builds the rows' axis-a vectors in LDS
// (thread-minor, conflict-free), then the four waves share the rows' 16-byte
// blocks (wave w: block indices w, w + 4, ..), so that a wave's stores of one
// block index are 1 KB in one piece and four waves keep stores in flight per
// set of vectors.  Which vector entries a block multiplies depends on the
// instance's box only: the workgroup tabulates it in LDS once per instance
// (a lane per block, K x D column indices, padding nodes pointing at a zero
// column), so the block loop reads one table entry and K x D vector values.
// The exit mass is accumulated axis by axis, exactly 0 when nothing leaves.
template <typename T, int D>
__global__ void __launch_bounds__(256) k_assemble_ell_sep(PlanDev P, int n,
                                                          const WorkItem *__restrict__ work,
                                                          int n_work, int lmax,
                                                          int *__restrict__ org,
                                                          T *__restrict__ vals,
                                                          T *__restrict__ exit_mass)
{
    constexpr int K = EllBlock<T>::K;
    static_assert(K * D <= 16, "a table entry holds the K x D column indices of a block");
    using B = EllBlock<T>;
    extern __shared__ unsigned char smem_raw[];
    // [D][value, slope][lmax][64], then the zero column zcol (host: zcol <= 255)
    T *vec = reinterpret_cast<T *>(smem_raw);
    const int zcol = D * 2 * lmax;
    // 16 bytes per block of the current instance: column of entry j, axis a at j D + a
    unsigned char *tab = smem_raw + (size_t)(zcol + 1) * 64 * sizeof(T);
    __shared__ T mass[2][3][64];                // per axis: inside, outside weight
    __shared__ int orgs[3][64];
    const T *w1 = weights1<T>(P);
    // the wave index as a uniform value: the block loop runs on the scalar unit
    const int t = threadIdx.x % 64, wv = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    auto V = [&](int a, int v, int l) -> T & { return vec[((a * 2 + v) * lmax + l) * 64 + t]; };
    if (threadIdx.x < 64) vec[zcol * 64 + threadIdx.x] = T(0);
    int cur = -1;   // instance the table holds
    const WorkRange wr = work_range(0, n_work);
    for (int w = wr.begin; w < wr.end; w += wr.step) {
        const WorkItem it = work[w];
        const DevInst &I = P.inst[it.inst];
        const int nbox = I.ell_w / (D + 1);
        const int bpf = I.ell_nbp / K;
        const int nblk = (D + 1) * bpf;
        if (it.inst != cur) {
            // blocks: field f (0 value, 1 + a slope along a), K box nodes each,
            // box nodes in order with the last axis fastest; padding nodes hold 0
            cur = it.inst;
            unsigned long long rb[3];
            for (int a = 0; a < D; ++a) rb[a] = fast_recip(I.ell_box[a]);
            for (int g = threadIdx.x; g < nblk; g += 256) {
                const int f = g / bpf;
                int l = (g - f * bpf) * K;
                int li[3] = {0, 0, 0};
                int rem = l;
                for (int a = D - 1; a >= 0; --a) {
                    const int q = fast_div(rem, rb[a]);
                    li[a] = rem - q * I.ell_box[a];
                    rem = q;
                }
                unsigned int e[4] = {0u, 0u, 0u, 0u};
                for (int j = 0; j < K; ++j, ++l) {
                    for (int a = 0; a < D; ++a) {
                        const unsigned int col = l < nbox
                            ? (unsigned int)((a * 2 + (f == a + 1 ? 1 : 0)) * lmax + li[a])
                            : (unsigned int)zcol;
                        const int k = j * D + a;
                        e[k / 4] |= col << (8 * (k % 4));
                    }
                    for (int a = D - 1; a >= 0; --a) {
                        if (++li[a] < I.ell_box[a]) break;
                        li[a] = 0;
                    }
                }
                *reinterpret_cast<uint4 *>(tab + (size_t)g * 16) = make_uint4(e[0], e[1], e[2], e[3]);
            }
        }
        const bool valid = t < it.count;
        const long long r = it.first + t;   // row within the instance
        const long long row = I.act_off + r;
        if (wv < D && valid) {
            const int a = wv;
            const int node = P.active[row];
            int idx[3];
            split_node<D>(I, node, idx);
            double c[3];
            node_centre<D>(I, P.coords, time_factors(P, n, it.inst), P.trig, idx, P.dt, c);
            const int L = I.ell_box[a];
            for (int l = 0; l < L; ++l) {
                V(a, 0, l) = T(0);
                V(a, 1, l) = T(0);
            }
            const int origin = eval_axis(I, P.coords, a, c[a], P.gh_a[0]).k;
            T in_a = T(0), out_a = T(0);
            // the landing cells rise with q (ascending GH nodes, S >= 0), so the
            // sums of the two nodes of the current cell stay in registers and
            // a node's total goes to LDS once, when the cell moves past it
            // (the same additions in the same order as accumulating in LDS)
            int wl = -1;                                 // cell of the window
            T v0 = T(0), d0 = T(0), v1 = T(0), d1 = T(0);   // nodes wl, wl + 1
            auto flush = [&](int node, T v, T d) {
                V(a, 0, node) += v;
                V(a, 1, node) += d;
            };
            for (int q = 0; q < P.qs; ++q) {
                const AxisEval e = eval_axis(I, P.coords, a, c[a], P.gh_a[q]);
                const T wq = w1[q];
                if (e.ex) {
                    out_a += wq;
                    continue;
                }
                const int l = e.k - origin;
                if (l < 0 || l + 1 >= L) {
                    atomicOr(P.flags, 2);
                    continue;
                }
                if (l != wl) {
                    if (wl >= 0) {
                        flush(wl, v0, d0);
                        if (l == wl + 1) {
                            v0 = v1;
                            d0 = d1;
                        } else {
                            flush(wl + 1, v1, d1);
                            v0 = T(0);
                            d0 = T(0);
                        }
                        v1 = T(0);
                        d1 = T(0);
                    }
                    wl = l;
                }
                const Basis<T> Bq = hermite<T>(e.s, e.h);
                v0 += wq * Bq.v0;
                v1 += wq * Bq.v1;
                d0 += wq * Bq.d0;
                d1 += wq * Bq.d1;
                in_a += wq;
            }
            if (wl >= 0) {
                flush(wl, v0, d0);
                flush(wl + 1, v1, d1);
            }
            mass[0][a][t] = in_a;
            mass[1][a][t] = out_a;
            orgs[a][t] = origin;
        }
        __syncthreads();
        if (valid) {
            if (wv == 0) {
                // mass of the tensor points with some axis outside, over axes 0..a
                T em = T(0), in_all = T(1);
                for (int a = 0; a < D; ++a) {
                    em = em * (mass[0][a][t] + mass[1][a][t]) + in_all * mass[1][a][t];
                    in_all *= mass[0][a][t];
                }
                for (int a = 0; a < 3; ++a) org[row * 3 + a] = a < D ? orgs[a][t] : 0;
                exit_mass[row] = em;
            }
            const long long rows = I.n_act;
            B *dst = reinterpret_cast<B *>(vals + I.ell_off) + r;
#pragma unroll 2
            for (int g = wv; g < nblk; g += 4) {
                const uint4 e4 = *reinterpret_cast<const uint4 *>(tab + (size_t)g * 16);
                const unsigned int e[4] = {e4.x, e4.y, e4.z, e4.w};
                T x[K][D];
#pragma unroll
                for (int j = 0; j < K; ++j)
#pragma unroll
                    for (int a = 0; a < D; ++a) {
                        const int k = j * D + a;
                        const unsigned int col = (e[k / 4] >> (8 * (k % 4))) & 255u;
                        x[j][a] = vec[col * 64 + t];
                    }
                B blk;
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    T v = x[j][0];
#pragma unroll
                    for (int a = 1; a < D; ++a) v *= x[j][a];
                    blk.v[j] = v;
                }
                store_block_nt(dst + (long long)g * rows, blk);
            }
        }
        __syncthreads();   // the vectors (and the table) are rebuilt for the next work item
    }
}

// Box-row product, one row per lane: the row walks its box nodes in order
// (coordinates advanced incrementally), gathering one node record per box
// node, and reads its values a 16-byte block (K box nodes of one field) at a
// time; blocks of one index are contiguous across the rows of the instance,
// so a wave's block load is 1 KB in one piece:
//   u^n[row] = uref + exit_mass[row] (1 - uref) + sum_box (v_u (u - uref) + sum_a v_a g_a),
// i.e. exit_mass + A [u; g] in offset form about uref = u^{n+1}[row].
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_ell_apply(PlanDev P, const int *__restrict__ org,
                                                      const T *__restrict__ vals,
                                                      const T *__restrict__ exit_mass,
                                                      const T *__restrict__ packed,
                                                      T *__restrict__ u_out)
{
    constexpr int PS = RecStride<D>::value;
    using R = typename RecT<T, PS>::type;
    const R *rec = reinterpret_cast<const R *>(packed);
    const WorkRange wr = work_range(0, P.n_row_work);
    for (int w = wr.begin; w < wr.end; w += wr.step) {
        const WorkItem it = P.row_work[w];
        if ((int)threadIdx.x >= it.count) continue;
        const DevInst &I = P.inst[it.inst];
        const long long rows = I.n_act;
        const long long r = it.first + threadIdx.x;
        const long long row = I.act_off + r;
        const int node = P.active[row];
        const T uref = rec[I.node_off + node].x;
        int o[3] = {0, 0, 0};
        for (int a = 0; a < D; ++a) o[a] = org[row * 3 + a];
        constexpr int K = EllBlock<T>::K;
        using B = EllBlock<T>;
        const int bpf = I.ell_nbp / K;
        const B *v0 = reinterpret_cast<const B *>(vals + I.ell_off) + r;
        const long long fs = (long long)bpf * rows;   // stride between field planes, in blocks
        T acc = exit_mass[row] * (T(1) - uref);
        int bi[3] = {0, 0, 0};
        for (int lb = 0; lb < bpf; ++lb) {
            const B *vp = v0 + (long long)lb * rows;
            B vf[D + 1];
#pragma unroll
            for (int f = 0; f <= D; ++f) vf[f] = vp[f * fs];
            // K independent gathers in flight per lane; past the last box node
            // the coordinates wrap to the origin (padding values are 0)
#pragma unroll
            for (int j = 0; j < K; ++j) {
                long long nd = I.node_off;
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    int ia = o[a] + bi[a];
                    if (ia > I.n[a] - 1) ia = I.n[a] - 1;   // zero-valued box nodes stay in range
                    nd += (long long)ia * I.stride[a];
                }
                const R rc = rec[nd];
                if constexpr (D == 1) {
                    acc += vf[0].v[j] * (rc.x - uref) + vf[1].v[j] * rc.y;
                } else if constexpr (D == 2) {
                    acc += vf[0].v[j] * (rc.x - uref) + vf[1].v[j] * rc.y + vf[2].v[j] * rc.z;
                } else {
                    acc += vf[0].v[j] * (rc.x - uref) + vf[1].v[j] * rc.y + vf[2].v[j] * rc.z +
                           vf[3].v[j] * rc.w;
                }
                // next box node (last axis fastest)
#pragma unroll
                for (int a = D - 1; a >= 0; --a) {
                    if (++bi[a] < I.ell_box[a]) break;
                    bi[a] = 0;
                }
            }
        }
        int idx[3];
        split_node<D>(I, node, idx);
        const T v = uref + acc;
        flag_nonfinite(P.flags, v);
        store_node<D, T>(I, idx, node, v, u_out);
    }
}

// Multi-column product (Algorithm 1): the assembled A_n applied to nc <= NC
// columns at once, a sparse matrix times a dense block.  Each row's value
// blocks are read once and contracted with the records of every column
// (column c's records at packed + c * plane, its field at u_out + c * fstride);
// the per-column arithmetic is that of k_ell_apply.
template <typename T, int D, int NC>
__global__ void __launch_bounds__(kBlock) k_ell_apply_mc(PlanDev P, const int *__restrict__ org,
                                                         const T *__restrict__ vals,
                                                         const T *__restrict__ exit_mass,
                                                         const T *__restrict__ packed,
                                                         long long plane, T *__restrict__ u_out,
                                                         long long fstride, int nc)
{
    constexpr int PS = RecStride<D>::value;
    using R = typename RecT<T, PS>::type;
    const R *rec = reinterpret_cast<const R *>(packed);
    const long long rplane = plane / PS;   // records between column planes
    const WorkRange wr = work_range(0, P.n_row_work);
    for (int w = wr.begin; w < wr.end; w += wr.step) {
        const WorkItem it = P.row_work[w];
        if ((int)threadIdx.x >= it.count) continue;
        const DevInst &I = P.inst[it.inst];
        const long long rows = I.n_act;
        const long long r = it.first + threadIdx.x;
        const long long row = I.act_off + r;
        const int node = P.active[row];
        const T em = exit_mass[row];
        T uref[NC], acc[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            uref[c] = c < nc ? rec[c * rplane + I.node_off + node].x : T(0);
            acc[c] = em * (T(1) - uref[c]);
        }
        int o[3] = {0, 0, 0};
        for (int a = 0; a < D; ++a) o[a] = org[row * 3 + a];
        constexpr int K = EllBlock<T>::K;
        using B = EllBlock<T>;
        const int bpf = I.ell_nbp / K;
        const B *v0 = reinterpret_cast<const B *>(vals + I.ell_off) + r;
        const long long fs = (long long)bpf * rows;
        int bi[3] = {0, 0, 0};
        for (int lb = 0; lb < bpf; ++lb) {
            const B *vp = v0 + (long long)lb * rows;
            B vf[D + 1];
#pragma unroll
            for (int f = 0; f <= D; ++f) vf[f] = vp[f * fs];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                long long nd = I.node_off;
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    int ia = o[a] + bi[a];
                    if (ia > I.n[a] - 1) ia = I.n[a] - 1;
                    nd += (long long)ia * I.stride[a];
                }
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    if (c >= nc) break;
                    const R rc = rec[c * rplane + nd];
                    if constexpr (D == 1) {
                        acc[c] += vf[0].v[j] * (rc.x - uref[c]) + vf[1].v[j] * rc.y;
                    } else if constexpr (D == 2) {
                        acc[c] += vf[0].v[j] * (rc.x - uref[c]) + vf[1].v[j] * rc.y + vf[2].v[j] * rc.z;
                    } else {
                        acc[c] += vf[0].v[j] * (rc.x - uref[c]) + vf[1].v[j] * rc.y +
                                  vf[2].v[j] * rc.z + vf[3].v[j] * rc.w;
                    }
                }
#pragma unroll
                for (int a = D - 1; a >= 0; --a) {
                    if (++bi[a] < I.ell_box[a]) break;
                    bi[a] = 0;
                }
            }
        }
        int idx[3];
        split_node<D>(I, node, idx);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (c >= nc) break;
            const T v = uref[c] + acc[c];
            flag_nonfinite(P.flags, v);
            store_node<D, T>(I, idx, node, v, u_out + c * fstride);
        }
    }
}

// Export in the documented layout: width P.ell_width (the largest instance
// width), column-major over all active rows, columns (d+1) node + field,
// padding entries value 0 (column of the row's own node value).
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_export_ell(PlanDev P, const int *org_in,
                                                       const T *vals_in, int *cols_out,
                                                       T *vals_out)
{
    const long long na = P.n_active;
    const long long total = na * (long long)P.ell_width;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
         t += (long long)gridDim.x * blockDim.x) {
        const int k = (int)(t / na);
        const long long row = t - (long long)k * na;
        // instance of the row (binary search over act_off)
        int lo = 0, hi = P.n_inst - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (P.inst[mid].act_off <= row) lo = mid; else hi = mid - 1;
        }
        const DevInst &I = P.inst[lo];
        const long long r = row - I.act_off;
        if (k < I.ell_w) {
            const int nbox = I.ell_w / (D + 1);
            const int f = k / nbox;
            int rest = k - f * nbox;
            long long nd = I.node_off;
            for (int a = D - 1; a >= 0; --a) {
                const int la = rest % I.ell_box[a];
                rest /= I.ell_box[a];
                int ia = org_in[row * 3 + a] + la;
                if (ia > I.n[a] - 1) ia = I.n[a] - 1;
                nd += (long long)ia * I.stride[a];
            }
            constexpr int K = EllBlock<T>::K;
            const int l = k - f * nbox;
            const long long blk = (long long)f * (I.ell_nbp / K) + l / K;
            cols_out[t] = (int)(nd * (D + 1) + f);
            vals_out[t] = vals_in[I.ell_off + (blk * I.n_act + r) * K + l % K];
        } else {
            cols_out[t] = (int)((I.node_off + P.active[row]) * (D + 1));
            vals_out[t] = T(0);
        }
    }
}

__global__ void k_clear_flags(int *flags) { flags[0] = 0; }

__global__ void __launch_bounds__(kBlock) k_zero(unsigned int *p, long long n)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// ---------------------------------------------------------------------------
// Adjoint (exit classification held fixed).  Step n: given lam^n on active
// nodes, scatter mu = A_n^T lam^n into per-node records (mu_u, mu_g...), and
// accumulate dJ/dtheta += lam^n_j sum_q w_q grad_z I(z_jq) . dz_jq/dtheta.
// ---------------------------------------------------------------------------
template <typename T, int D, int G>
__global__ void __launch_bounds__(kBlock) k_adjoint_step(PlanDev P, int n,
                                                         const T *__restrict__ packed,
                                                         const T *__restrict__ lam,
                                                         T *__restrict__ mu,
                                                         double *__restrict__ grad)
{
    constexpr int PS = RecStride<D>::value;
    using R = typename RecT<T, PS>::type;
    const R *rec = reinterpret_cast<const R *>(packed);
    const T *W = weights<T>(P);
    const int lane = threadIdx.x % G;
    const int slot = threadIdx.x / G;
    __shared__ double red[kBlock / 64][kThetaSlots];
    const WorkRange wr = work_range(0, P.n_act_work);
    for (int w = wr.begin; w < wr.end; w += wr.step) {
        const WorkItem it = P.act_work[w];
        const bool valid = slot < it.count;
        const DevInst &I = P.inst[it.inst];
        double gth[kThetaSlots];
        for (int k = 0; k < kThetaSlots; ++k) gth[k] = 0.0;
        if (valid) {
            const int node = P.active[I.act_off + it.first + slot];
            int idx[3];
            split_node<D>(I, node, idx);
            const T L = lam[I.node_off + node];
            if (L != T(0)) {
                const double *tf = time_factors(P, n, it.inst);
                double c[3];
                node_centre<D>(I, P.coords, tf, P.trig, idx, P.dt, c);
                // per axis: sum_q w_q dI/dz_a and sum_q w_q a_{q_a} dI/dz_a
                T Gz[3] = {T(0), T(0), T(0)}, Hz[3] = {T(0), T(0), T(0)};
                for (int q = lane; q < P.n_quad; q += G) {
                    int k[3];
                    double s[3], h[3];
                    if (landing_point<D>(I, P.coords, P.gh_a, P.qs, c, q, k, s, h)) continue;
                    const T wq = W[q];
                    const T Lw = L * wq;
                    Basis<T> B[3], Bz[3];
                    for (int a = 0; a < D; ++a) {
                        B[a] = hermite<T>(s[a], h[a]);
                        Bz[a] = hermite_dz<T>(s[a], h[a]);
                    }
                    R p[1 << D];
                    gather_corners<D, R>(rec, I, k, p);
                    T gz[3];
                    hermite_grad<T, D, R>(p, B, Bz, gz);
                    int qr = q, qi[3];
                    for (int a = D - 1; a >= 0; --a) { qi[a] = qr % P.qs; qr /= P.qs; }
                    for (int a = 0; a < D; ++a) {
                        Gz[a] += wq * gz[a];
                        Hz[a] += wq * (T)P.gh_a[qi[a]] * gz[a];
                    }
                    // scatter the transposed row into mu
                    long long base = I.node_off;
                    for (int a = 0; a < D; ++a) base += (long long)k[a] * I.stride[a];
                    for (int cb = 0; cb < (1 << D); ++cb) {
                        long long o = base;
                        T wv = Lw;
                        for (int a = 0; a < D; ++a) {
                            const int bit = (cb >> (D - 1 - a)) & 1;
                            o += bit * I.stride[a];
                            wv *= bit ? B[a].v1 : B[a].v0;
                        }
                        atomicAdd(&mu[o * PS], wv);
                        for (int a = 0; a < D; ++a) {
                            T ws = Lw;
                            for (int i = 0; i < D; ++i) {
                                const int bit = (cb >> (D - 1 - i)) & 1;
                                if (i == a) ws *= bit ? B[i].d1 : B[i].d0;
                                else ws *= bit ? B[i].v1 : B[i].v0;
                            }
                            atomicAdd(&mu[o * PS + 1 + a], ws);
                        }
                    }
                }
                double db[12];
                const int nt = drift_dtheta<D>(I, tf, P.trig, idx, db);
                for (int kk = 0; kk < nt; ++kk) {
                    double sdot = 0.0;
                    for (int a = 0; a < D; ++a) sdot += (double)Gz[a] * db[kk * 3 + a];
                    gth[kk] = (double)L * P.dt * sdot;
                }
                double sd = 0.0;
                for (int a = 0; a < D; ++a) sd += (double)Hz[a];
                gth[nt] = (double)L * sd * I.dSdD;
            }
        }
        // block reduction of the parameter gradient, one atomic per entry
        const int wave = threadIdx.x / 64, wl = threadIdx.x % 64;
        for (int kk = 0; kk < kThetaSlots; ++kk) {
            double v = gth[kk];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (wl == 0) red[wave][kk] = v;
        }
        __syncthreads();
        if (threadIdx.x < kThetaSlots) {
            double v = 0.0;
            for (int wv = 0; wv < kBlock / 64; ++wv) v += red[wv][threadIdx.x];
            if (v != 0.0) atomicAdd(&grad[it.inst * kThetaSlots + threadIdx.x], v);
        }
        __syncthreads();
    }
}


// LDS accumulator (FP64) of mu for one work item: D + 1 field planes (value, then the
// slope along each axis), each a box of nodes [lo, lo + ext) with the
// innermost axis padded to `pitch` entries (host-chosen so that the rows of a
// wave's patch fall on distinct banks).  Entries outside the box, or every
// entry when the box does not fit (use == false), go to global memory.
template <typename T, int D>
struct MuTile {
    static constexpr int NF = D + 1;
    double *lds;
    int lo[3], ext[3];
    int pitch, plane, total;
    // reciprocals for the flush's index decoding: floor(n / d) = (n m) >> 32
    // with m = floor(2^32 / d) + 1, exact while n d < 2^32 (tiles hold fewer
    // than 2^13 entries)
    unsigned long long rplane, rpitch, rext1, rlast;
    int soff, cells;
    bool use;

    __device__ static unsigned long long recip(int d)
    {
        return (1ull << 32) / (unsigned long long)d + 1ull;
    }
    __device__ static int qdiv(int n, unsigned long long m)
    {
        return (int)(((unsigned long long)(unsigned)n * m) >> 32);
    }

    __device__ void init(double *mem, const TileBox &tb)
    {
        lds = mem;
        use = tb.use_lds != 0;
        plane = 1;
        for (int a = 0; a < 3; ++a) {
            lo[a] = tb.lo[a];
            ext[a] = tb.ext[a];
        }
        pitch = tb.pad;
        for (int a = 0; a < D - 1; ++a) plane *= ext[a];
        plane *= pitch;
        total = NF * plane;
        rplane = recip(plane);
        rpitch = recip(pitch);
        rext1 = recip(ext[1] > 0 ? ext[1] : 1);
        rlast = recip(ext[D - 1]);
        soff = tb.soff;
        cells = plane / pitch * ext[D - 1];
    }

    __device__ void clear() const
    {
        if (use)
            for (int e = threadIdx.x; e < total; e += blockDim.x) lds[e] = 0.0;
    }

    // plane offset of the cell whose lowest corner is k when all 2^D corners
    // lie in the box, else -1
    __device__ int cell_offset(const int *k) const
    {
        if (!use) return -1;
        int off = 0;
        bool in = true;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const int l = k[a] - lo[a];
            in = in && l >= 0 && l + 1 < ext[a];
            off = (a == D - 1) ? off * pitch + l : off * ext[a] + l;
        }
        return in ? off : -1;
    }

    // plane offset of one node, or -1 outside the box
    __device__ int node_offset(const int *k) const
    {
        if (!use) return -1;
        int off = 0;
        bool in = true;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const int l = k[a] - lo[a];
            in = in && l >= 0 && l < ext[a];
            off = (a == D - 1) ? off * pitch + l : off * ext[a] + l;
        }
        return in ? off : -1;
    }

    // add the tile to mu (node records of stride PS): with plain stores into
    // the tile's staging slot (every entry, fields interleaved; k_gather_tiles
    // sums the slots per node), else with global atomics
    template <int PS>
    __device__ void flush(const DevInst &I, T *mu, T *stage) const
    {
        if (!use) return;
        if (stage != nullptr && soff >= 0) {
            // slot order (cell, field): consecutive lanes store consecutive words
            T *slot = stage + soff;
            for (int k = threadIdx.x; k < cells * NF; k += blockDim.x) {
                const int c = k / NF, f = k - c * NF;
                const int row = qdiv(c, rlast), ll = c - row * ext[D - 1];
                slot[k] = (T)lds[f * plane + row * pitch + ll];
            }
            return;
        }
        for (int e = threadIdx.x; e < total; e += blockDim.x) {
            const T v = (T)lds[e];
            if (v == T(0)) continue;
            // e = ((f ext0 + l0) ext1 + l1) pitch + ll in 3D, (f ext0 + l0) pitch + ll in 2D
            const int f = qdiv(e, rplane);
            const int r = e - f * plane;
            const int row = qdiv(r, rpitch);
            const int ll = r - row * pitch;
            if (ll >= ext[D - 1]) continue;
            // tiles of periodic axes may run past the seam: wrap back onto the grid
            long long o = I.node_off + (long long)wrap_index(lo[D - 1] + ll, I.n[D - 1],
                                                             I.periodic[D - 1]) * I.stride[D - 1];
            if constexpr (D == 2) {
                o += (long long)wrap_index(lo[0] + row, I.n[0], I.periodic[0]) * I.stride[0];
            } else if constexpr (D == 3) {
                const int l0 = qdiv(row, rext1), l1 = row - l0 * ext[1];
                o += (long long)wrap_index(lo[1] + l1, I.n[1], I.periodic[1]) * I.stride[1];
                o += (long long)wrap_index(lo[0] + l0, I.n[0], I.periodic[0]) * I.stride[0];
            }
            atomicAdd(&mu[o * PS + f], v);
        }
    }
};

// Reduce per-lane theta-gradient terms over the workgroup and add them to the
// instance's slots (one atomic per slot and work item).
__device__ inline void reduce_theta(double (*red)[kThetaSlots], const double *gth,
                                    double *grad, int inst)
{
    const int wave = threadIdx.x / 64, wl = threadIdx.x % 64;
    for (int kk = 0; kk < kThetaSlots; ++kk) {
        double v = gth[kk];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (wl == 0) red[wave][kk] = v;
    }
    __syncthreads();
    if (threadIdx.x < kThetaSlots) {
        double v = 0.0;
        for (int wv = 0; wv < kBlock / 64; ++wv) v += red[wv][threadIdx.x];
        if (v != 0.0) atomicAdd(&grad[inst * kThetaSlots + threadIdx.x], v);
    }
}

// mu += the staged tile entries that cover each node (fixed order: the tiles'
// order in the work lists), after the transposed-step kernels.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_gather_tiles(int n_cov, const int *__restrict__ cov_node,
                                                         const int *__restrict__ cov_ptr,
                                                         const int *__restrict__ cov_base,
                                                         const T *__restrict__ stage,
                                                         T *__restrict__ mu)
{
    constexpr int NF = D + 1, PS = RecStride<D>::value;
    const int stride = gridDim.x * blockDim.x;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n_cov; t += stride) {
        const long long j = cov_node[t];
        const int b = cov_ptr[t], e = cov_ptr[t + 1];
        T acc[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) acc[f] = T(0);
        for (int k = b; k < e; ++k) {
            const T *sp = stage + cov_base[k];
#pragma unroll
            for (int f = 0; f < NF; ++f) acc[f] += sp[f];
        }
#pragma unroll
        for (int f = 0; f < NF; ++f)
            if (acc[f] != T(0)) mu[j * PS + f] += acc[f];
    }
}

// theta-gradient of one node from the weighted interpolant gradients:
// Gz = sum_q w_q grad I(z_q), Hz = sum_q w_q a_q . grad I(z_q).
template <int D, typename T>
__device__ inline void node_theta(const PlanDev &P, const DevInst &I, const double *tf,
                                  const double2 *trig, const int *idx, T Lm, const T *Gz,
                                  const T *Hz, double *gth)
{
    double db[12];
    const int nt = drift_dtheta<D>(I, tf, trig, idx, db);
    double sd = 0.0;
    for (int a = 0; a < D; ++a) sd += (double)Hz[a];
    const double gD = (double)Lm * sd * I.dSdD;
    // constant indices only, so that gth and db stay in registers
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        double sdot = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) sdot += (double)Gz[a] * db[kk * 3 + a];
        gth[kk] = kk < nt ? (double)Lm * P.dt * sdot : (kk == nt ? gD : 0.0);
    }
    gth[4] = nt == 4 ? gD : 0.0;
}

// Thread-per-node adjoint step.  Lane = active node.  For each inside landing
// point the kernel adds the transposed interpolation weights (2^D corners x
// (value, D slopes)) times lam_j w_q to mu, and accumulates the interpolant's
// gradient for the theta-derivative.  The innermost axis' landing data (cell,
// in-cell position, width, exit flag, ball distance) are evaluated once per
// node; the Hermite bases are rebuilt from them per point, which keeps the
// kernel's registers low enough for several waves per SIMD.  The scatter goes
// to the work item's LDS tile (field planes, padded rows), flushed once.  IN
// (2D): the host has shown that no landing point of the work item's nodes can
// exit (reach bound), so the exit tests and their per-point data are left out.
template <typename T, int D, int QS, bool AFF, bool IN>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 3 : 2))) k_adjoint_node(
    const PlanDev P, int n, int n_work, const DevInst *__restrict__ insts,
    const WorkItem *__restrict__ work, const TileBox *__restrict__ tiles,
    const int *__restrict__ nodes, const double2 *__restrict__ trig,
    const double *__restrict__ coords, const T *__restrict__ packed,
    const T *__restrict__ lam, T *__restrict__ mu, double *__restrict__ grad)
{
    constexpr int PS = RecStride<D>::value;
    using R = typename RecT<T, PS>::type;
    extern __shared__ unsigned char smem_raw[];
    __shared__ double red[kBlock / 64][kThetaSlots];
    const R *rec = reinterpret_cast<const R *>(packed);
    const double *ga = P.gh_a;
    const T *w1 = weights1<T>(P);
    const WorkRange wr = work_range(0, n_work);
    for (int w = wr.begin; w < wr.end; w += wr.step) {
        const WorkItem it = work[w];
        const DevInst &I = insts[it.inst];
        double *const tmem = reinterpret_cast<double *>(smem_raw);
        MuTile<T, D> tile;
        tile.init(tmem, tiles[w]);
        tile.clear();
        __syncthreads();
        double gth[kThetaSlots];
        for (int kk = 0; kk < kThetaSlots; ++kk) gth[kk] = 0.0;
        const bool valid = (int)threadIdx.x < it.count;
        const int node = valid ? nodes[it.first + threadIdx.x] : 0;
        const T Lm = valid ? lam[I.node_off + node] : T(0);
        if (valid && Lm != T(0)) {
            int idx[3];
            split_node<D>(I, node, idx);
            const double *tf = time_factors(P, n, it.inst);
            double c[3];
            node_centre<D>(I, coords, tf, trig, idx, P.dt, c);
            const bool ball = I.region_kind == 1;
            const double r2 = I.r2;
            constexpr int AI = D - 1;
            int kin[QS];
            T sin_[QS], hin[QS];
            bool exin[QS];
            double din[QS];
#pragma unroll
            for (int q = 0; q < QS; ++q) {
                const AxisEval e = eval_axis_t<AFF>(I, coords, AI, c[AI], ga[q]);
                kin[q] = e.k;
                sin_[q] = (T)e.s;
                hin[q] = (T)e.h;
                exin[q] = e.ex;
                din[q] = e.dz2;
            }
            T Gz[3] = {T(0), T(0), T(0)}, Hz[3] = {T(0), T(0), T(0)};
            if constexpr (D == 2) {
                const long long s0 = I.stride[0];
                const int pl = tile.plane, pitch = tile.pitch;
                // one row of landing points at a time (unrolled rows would hold
                // every row's gathers in registers)
#pragma unroll 1
                for (int q0 = 0; q0 < QS; ++q0) {
                    const AxisEval e0 = eval_axis_t<AFF>(I, coords, 0, c[0], ga[q0]);
                    if (!IN && e0.ex) continue;
                    const Basis<T> X = hermite<T>(e0.s, e0.h), Xz = hermite_dz<T>(e0.s, e0.h);
                    const T w0 = w1[q0], a0 = (T)ga[q0];
                    const T Lw0 = Lm * w0;
                    // the row's LDS offset (cell k0, innermost cell 0) when the
                    // whole row of cells k0 fits the tile along axis 0
                    const int l0 = e0.k - tile.lo[0];
                    const bool row_in = tile.use && l0 >= 0 && l0 + 1 < tile.ext[0];
                    const int row_off = l0 * pitch - tile.lo[1];
                    const long long row = I.node_off + (long long)e0.k * s0;
#pragma unroll
                    for (int q1 = 0; q1 < QS; ++q1) {
                        if constexpr (!IN) {
                            bool ex = exin[q1];
                            if (ball) ex = ex || ball_exit2(e0.dz2, din[q1], r2);
                            if (ex) continue;
                        }
                        T s = sin_[q1], h = hin[q1];
                        // the bases below depend on q1 only: keep them from being
                        // hoisted out of the q0 loop for all q1 at once (that
                        // would hold 8 x 12 values in registers and spill)
                        int k1 = kin[q1];
                        asm volatile("" : "+v"(s), "+v"(h), "+v"(k1));
                        // interior points have valid cells; the (never taken)
                        // branch keeps each point's code in its own block
                        if (IN && k1 < 0) continue;
                        const T om = T(1) - s;
                        const T yv0 = (T(1) + T(2) * s) * om * om, yv1 = s * s * (T(3) - T(2) * s);
                        const T yd0 = h * s * om * om, yd1 = h * s * s * (s - T(1));
                        const T zv0 = (T(6) * s * s - T(6) * s) / h, zv1 = (T(6) * s - T(6) * s * s) / h;
                        const T zd0 = T(1) - T(4) * s + T(3) * s * s, zd1 = T(3) * s * s - T(2) * s;
                        const long long b = row + k1;
                        const R p00 = rec[b], p01 = rec[b + 1], p10 = rec[b + s0], p11 = rec[b + s0 + 1];
                        // interpolant gradient: d/dz0 (Xz, Y) and d/dz1 (X, Yz)
                        const T A0z = p00.x * Xz.v0 + p10.x * Xz.v1 + p00.y * Xz.d0 + p10.y * Xz.d1;
                        const T A1z = p01.x * Xz.v0 + p11.x * Xz.v1 + p01.y * Xz.d0 + p11.y * Xz.d1;
                        const T C0z = p00.z * Xz.v0 + p10.z * Xz.v1;
                        const T C1z = p01.z * Xz.v0 + p11.z * Xz.v1;
                        const T g0 = yv0 * A0z + yv1 * A1z + yd0 * C0z + yd1 * C1z;
                        const T A0 = p00.x * X.v0 + p10.x * X.v1 + p00.y * X.d0 + p10.y * X.d1;
                        const T A1 = p01.x * X.v0 + p11.x * X.v1 + p01.y * X.d0 + p11.y * X.d1;
                        const T C0 = p00.z * X.v0 + p10.z * X.v1;
                        const T C1 = p01.z * X.v0 + p11.z * X.v1;
                        const T g1 = zv0 * A0 + zv1 * A1 + zd0 * C0 + zd1 * C1;
                        const T wq = w0 * w1[q1];
                        Gz[0] += wq * g0;
                        Gz[1] += wq * g1;
                        Hz[0] += wq * a0 * g0;
                        Hz[1] += wq * (T)ga[q1] * g1;
                        // transposed weights: corner (e0, e1) gets
                        // value X.v Y.v, slope-0 X.d Y.v, slope-1 X.v Y.d
                        const T w1q = Lw0 * w1[q1];
                        const T v0 = w1q * yv0, v1 = w1q * yv1, d0 = w1q * yd0, d1 = w1q * yd1;
                        const T e00 = X.v0 * v0, e01 = X.v0 * v1, e10 = X.v1 * v0, e11 = X.v1 * v1;
                        const T f00 = X.d0 * v0, f01 = X.d0 * v1, f10 = X.d1 * v0, f11 = X.d1 * v1;
                        const T g00 = X.v0 * d0, g01 = X.v0 * d1, g10 = X.v1 * d0, g11 = X.v1 * d1;
                        const int l1 = k1 - tile.lo[1];
                        if (row_in && l1 >= 0 && l1 + 1 < tile.ext[1]) {
                            double *t = tmem + row_off + k1;
                            lds_add(t, e00);
                            lds_add(t + 1, e01);
                            lds_add(t + pitch, e10);
                            lds_add(t + pitch + 1, e11);
                            t += pl;
                            lds_add(t, f00);
                            lds_add(t + 1, f01);
                            lds_add(t + pitch, f10);
                            lds_add(t + pitch + 1, f11);
                            t += pl;
                            lds_add(t, g00);
                            lds_add(t + 1, g01);
                            lds_add(t + pitch, g10);
                            lds_add(t + pitch + 1, g11);
                        } else {
                            T *m = mu + b * PS;
                            const long long sp = s0 * PS;
                            atomicAdd(m, e00);
                            atomicAdd(m + PS, e01);
                            atomicAdd(m + sp, e10);
                            atomicAdd(m + sp + PS, e11);
                            atomicAdd(m + 1, f00);
                            atomicAdd(m + PS + 1, f01);
                            atomicAdd(m + sp + 1, f10);
                            atomicAdd(m + sp + PS + 1, f11);
                            atomicAdd(m + 2, g00);
                            atomicAdd(m + PS + 2, g01);
                            atomicAdd(m + sp + 2, g10);
                            atomicAdd(m + sp + PS + 2, g11);
                        }
                    }
                }
            } else {
                // d = 1 and d = 3: one landing point at a time
                auto point = [&](const int *k, const Basis<T> *B, const Basis<T> *Bz, const T *aq, T wq) {
                    R p[1 << D];
                    gather_corners<D, R>(rec, I, k, p);
                    T gz[3];
                    hermite_grad<T, D, R>(p, B, Bz, gz);
                    for (int a = 0; a < D; ++a) {
                        Gz[a] += wq * gz[a];
                        Hz[a] += wq * aq[a] * gz[a];
                    }
                    const T Lw = Lm * wq;
                    // transposed weights: corner cb, field f (value, then the
                    // slope along axis f - 1, whose basis swaps to the slope one)
                    constexpr int NC = 1 << D;
                    T vals[NC][D + 1];
#pragma unroll
                    for (int cb = 0; cb < NC; ++cb) {
#pragma unroll
                        for (int f = 0; f <= D; ++f) {
                            T v = Lw;
#pragma unroll
                            for (int i = 0; i < D; ++i) {
                                const int bi = (cb >> (D - 1 - i)) & 1;
                                if (f == i + 1) v *= bi ? B[i].d1 : B[i].d0;
                                else v *= bi ? B[i].v1 : B[i].v0;
                            }
                            vals[cb][f] = v;
                        }
                    }
                    const int co = tile.cell_offset(k);
                    if (co >= 0) {
#pragma unroll
                        for (int cb = 0; cb < NC; ++cb) {
                            int loff = co;
#pragma unroll
                            for (int a = 0; a < D; ++a)
                                if ((cb >> (D - 1 - a)) & 1) {
                                    int st = 1;
                                    if (a < D - 1) {
                                        st = tile.pitch;
                                        for (int a2 = a + 1; a2 < D - 1; ++a2) st *= tile.ext[a2];
                                    }
                                    loff += st;
                                }
#pragma unroll
                            for (int f = 0; f <= D; ++f) lds_add(tmem + f * tile.plane + loff, vals[cb][f]);
                        }
                    } else {
                        long long gbase = I.node_off;
                        for (int a = 0; a < D; ++a) gbase += (long long)k[a] * I.stride[a];
#pragma unroll
                        for (int cb = 0; cb < NC; ++cb) {
                            long long goff = gbase;
#pragma unroll
                            for (int a = 0; a < D; ++a)
                                if ((cb >> (D - 1 - a)) & 1) goff += I.stride[a];
#pragma unroll
                            for (int f = 0; f <= D; ++f) atomicAdd(mu + goff * PS + f, vals[cb][f]);
                        }
                    }
                };
                if constexpr (D == 1) {
#pragma unroll
                    for (int q = 0; q < QS; ++q) {
                        if (exin[q] || (ball && din[q] >= r2)) continue;
                        int k[1] = {kin[q]};
                        const Basis<T> B = hermite<T>(sin_[q], hin[q]);
                        const Basis<T> Bz = hermite_dz<T>(sin_[q], hin[q]);
                        const T aq[1] = {(T)ga[q]};
                        point(k, &B, &Bz, aq, w1[q]);
                    }
                } else {
                    for (int q0 = 0; q0 < QS; ++q0) {
                        const AxisEval e0 = eval_axis_t<AFF>(I, coords, 0, c[0], ga[q0]);
                        if (e0.ex) continue;
                        const Basis<T> X = hermite<T>(e0.s, e0.h), dX = hermite_dz<T>(e0.s, e0.h);
                        for (int q1 = 0; q1 < QS; ++q1) {
                            const AxisEval e1 = eval_axis_t<AFF>(I, coords, 1, c[1], ga[q1]);
                            if (e1.ex) continue;
                            const Basis<T> Y = hermite<T>(e1.s, e1.h), dY = hermite_dz<T>(e1.s, e1.h);
#pragma unroll
                            for (int q2 = 0; q2 < QS; ++q2) {
                                if (exin[q2]) continue;
                                if (ball) {
                                    const double dz[3] = {e0.dz2, e1.dz2, din[q2]};
                                    if (ball_exit(dz, 3, r2)) continue;
                                }
                                int k[3] = {e0.k, e1.k, kin[q2]};
                                const Basis<T> Z = hermite<T>(sin_[q2], hin[q2]);
                                const Basis<T> dZ = hermite_dz<T>(sin_[q2], hin[q2]);
                                const Basis<T> B[3] = {X, Y, Z}, Bz[3] = {dX, dY, dZ};
                                const T aq[3] = {(T)ga[q0], (T)ga[q1], (T)ga[q2]};
                                point(k, B, Bz, aq, w1[q0] * w1[q1] * w1[q2]);
                            }
                        }
                    }
                }
            }
            node_theta<D, T>(P, I, tf, trig, idx, Lm, Gz, Hz, gth);
        }
        __syncthreads();
        tile.template flush<PS>(I, mu, (T *)P.adj.stage);
        reduce_theta(red, gth, grad, it.inst);
        __syncthreads();
    }
}

// Box-form adjoint step in 2D for separable nodes (affine axes).  The
// transposed row of A_n over the footprint box [o0, o0+L) x [o1, o1+L) is
// the outer product of the per-axis weight vectors: entry (i, j) gets
// lam_j (V0[i] V1[j], S0[i] V1[j], V0[i] S1[j]) for (value, slope-0, slope-1),
// i.e. 3 L^2 scatter adds per node against 12 per landing point in the
// per-point form.  The theta-gradient is the same box contraction of the
// records with the derivative vectors (dV, dS: z-derivative bases; aV, aS:
// the same times the GH node) on one axis at a time.  The axis-1 vectors live
// in registers; the axis-0 entries of row i are rebuilt inside the (rolled)
// row loop from the hoisted axis-0 landing data, which keeps the registers
// within a few waves per SIMD for L up to 12.
template <typename T, int QS, int L>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 1 : (L <= 8 ? 3 : 2)))) k_adjoint_box2(
    const PlanDev P, int n, int n_work, const DevInst *__restrict__ insts,
    const WorkItem *__restrict__ work, const TileBox *__restrict__ tiles,
    const int *__restrict__ nodes, const double2 *__restrict__ trig,
    const double *__restrict__ coords, const T *__restrict__ packed,
    const T *__restrict__ lam, T *__restrict__ mu, double *__restrict__ grad)
{
    constexpr int D = 2;
    constexpr int PS = RecStride<D>::value;
    using R = typename RecT<T, PS>::type;
    extern __shared__ unsigned char smem_raw[];
    __shared__ double red[kBlock / 64][kThetaSlots];
    const R *rec = reinterpret_cast<const R *>(packed);
    const double *ga = P.gh_a;
    const T *w1 = weights1<T>(P);
    const WorkRange wr = work_range(0, n_work);
    for (int w = wr.begin; w < wr.end; w += wr.step) {
        const WorkItem it = work[w];
        const DevInst &I = insts[it.inst];
        double *const tmem = reinterpret_cast<double *>(smem_raw);
        MuTile<T, D> tile;
        tile.init(tmem, tiles[w]);
        tile.clear();
        __syncthreads();
        double gth[kThetaSlots];
        for (int kk = 0; kk < kThetaSlots; ++kk) gth[kk] = 0.0;
        const bool valid = (int)threadIdx.x < it.count;
        const int node = valid ? nodes[it.first + threadIdx.x] : 0;
        const T Lm = valid ? lam[I.node_off + node] : T(0);
        if (valid && Lm != T(0)) {
            int idx[3];
            split_node<D>(I, node, idx);
            const double *tf = time_factors(P, n, it.inst);
            double c[3];
            node_centre<D>(I, coords, tf, trig, idx, P.dt, c);
            // axis 1: weight vectors over the footprint
            T V1[L], S1[L], dV1[L], dS1[L], aV1[L], aS1[L];
            int o1;
            T m1;
            bool ok = axis_vectors<T, QS, L, true, true>(I, coords, ga, w1, 1, c[1], o1, m1, V1, S1,
                                                         dV1, dS1, aV1, aS1);
            // axis 0: landing data per GH node
            int l0[QS];
            T s0[QS];
            bool in0[QS];
            int o0 = 0;
            T h0 = T(1);
#pragma unroll
            for (int q = 0; q < QS; ++q) {
                int ku;
                const AxisEval e = eval_axis_unwrapped<true>(I, coords, 0, c[0], ga[q], ku);
                if (q == 0) {
                    o0 = ku;
                    h0 = (T)e.h;
                }
                l0[q] = ku - o0;
                s0[q] = (T)e.s;
                in0[q] = !e.ex;
                ok = ok && l0[q] >= 0 && l0[q] <= L - 2;
            }
            if (!ok) atomicOr(P.flags, 2);
            const int b0 = o0 - tile.lo[0], b1 = o1 - tile.lo[1];
            const bool lds = tile.use && b0 >= 0 && b0 + L <= tile.ext[0] && b1 >= 0 &&
                             b1 + L <= tile.ext[1];
            T Gz0 = T(0), Gz1 = T(0), Hz0 = T(0), Hz1 = T(0);
            for (int i = 0; i < L; ++i) {
                // axis-0 entries of row o0 + i
                T v0 = T(0), sv0 = T(0), dv0 = T(0), ds0 = T(0), av0 = T(0), as0 = T(0);
                bool hit = false;
#pragma unroll
                for (int q = 0; q < QS; ++q) {
                    const bool lo = l0[q] == i, hi = l0[q] + 1 == i;
                    if (!in0[q] || !(lo || hi)) continue;
                    hit = true;
                    // the bases depend on q only: rebuilt per row rather than hoisted
                    // out of the row loop for every q at once (registers)
                    T sq = s0[q];
                    asm volatile("" : "+v"(sq));
                    const Basis<T> B = hermite<T>(sq, h0), Bz = hermite_dz<T>(sq, h0);
                    const T wq = w1[q], wa = wq * (T)ga[q];
                    v0 += wq * (lo ? B.v0 : B.v1);
                    sv0 += wq * (lo ? B.d0 : B.d1);
                    dv0 += wq * (lo ? Bz.v0 : Bz.v1);
                    ds0 += wq * (lo ? Bz.d0 : Bz.d1);
                    av0 += wa * (lo ? Bz.v0 : Bz.v1);
                    as0 += wa * (lo ? Bz.d0 : Bz.d1);
                }
                if (!hit) continue;
                const int ci = wrap_index(o0 + i, I.n[0], I.periodic[0]);
                const long long row = I.node_off + (long long)ci * I.stride[0];
                const T lv0 = Lm * v0, lsv0 = Lm * sv0;
                T tA = T(0), tB = T(0), tC = T(0), tD = T(0), tE = T(0), tF = T(0);
                if (lds) {
                    double *t = tmem + (b0 + i) * tile.pitch + b1;
#pragma unroll
                    for (int j = 0; j < L; ++j) {
                        const R r = rec[row + o1 + j];
                        tA += V1[j] * r.x + S1[j] * r.z;
                        tB += V1[j] * r.y;
                        tC += dV1[j] * r.x + dS1[j] * r.z;
                        tD += dV1[j] * r.y;
                        tE += aV1[j] * r.x + aS1[j] * r.z;
                        tF += aV1[j] * r.y;
                        lds_add(t + j, lv0 * V1[j]);
                        lds_add(t + tile.plane + j, lsv0 * V1[j]);
                        lds_add(t + 2 * tile.plane + j, lv0 * S1[j]);
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < L; ++j) {
                        const int cj = wrap_index(o1 + j, I.n[1], I.periodic[1]);
                        const R r = rec[row + cj];
                        tA += V1[j] * r.x + S1[j] * r.z;
                        tB += V1[j] * r.y;
                        tC += dV1[j] * r.x + dS1[j] * r.z;
                        tD += dV1[j] * r.y;
                        tE += aV1[j] * r.x + aS1[j] * r.z;
                        tF += aV1[j] * r.y;
                        T *m = mu + (row + cj) * PS;
                        atomicAdd(m, lv0 * V1[j]);
                        atomicAdd(m + 1, lsv0 * V1[j]);
                        atomicAdd(m + 2, lv0 * S1[j]);
                    }
                }
                Gz0 += dv0 * tA + ds0 * tB;
                Hz0 += av0 * tA + as0 * tB;
                Gz1 += v0 * tC + sv0 * tD;
                Hz1 += v0 * tE + sv0 * tF;
            }
            const T Gz[3] = {Gz0, Gz1, T(0)}, Hz[3] = {Hz0, Hz1, T(0)};
            node_theta<D, T>(P, I, tf, trig, idx, Lm, Gz, Hz, gth);
        }
        __syncthreads();
        tile.template flush<PS>(I, mu, (T *)P.adj.stage);
        reduce_theta(red, gth, grad, it.inst);
        __syncthreads();
    }
}

// Box-form adjoint step for separable nodes: the transposed row of A_n is the
// outer product of the per-axis weight vectors, and the theta-gradient needs
// the same box contraction with the derivative vectors (dV, dS) and the
// GH-node-weighted derivative vectors (aV, aS) on one axis at a time.
template <typename T, int D, int QS, int L, bool AFF>
__global__ void __launch_bounds__(kBlock) k_adjoint_box(
    const PlanDev P, int n, int n_work, const DevInst *__restrict__ insts,
    const WorkItem *__restrict__ work, const TileBox *__restrict__ tiles,
    const int *__restrict__ nodes, const double2 *__restrict__ trig,
    const double *__restrict__ coords, const T *__restrict__ packed,
    const T *__restrict__ lam, T *__restrict__ mu, double *__restrict__ grad)
{
    constexpr int PS = RecStride<D>::value;
    using R = typename RecT<T, PS>::type;
    extern __shared__ unsigned char smem_raw[];
    __shared__ double red[kBlock / 64][kThetaSlots];
    const R *rec = reinterpret_cast<const R *>(packed);
    const double *ga = P.gh_a;
    const T *w1 = weights1<T>(P);
    const WorkRange wr = work_range(0, n_work);
    for (int w = wr.begin; w < wr.end; w += wr.step) {
        const WorkItem it = work[w];
        const DevInst &I = insts[it.inst];
        double *const tmem = reinterpret_cast<double *>(smem_raw);
        MuTile<T, D> tile;
        tile.init(tmem, tiles[w]);
        tile.clear();
        __syncthreads();
        // uidx: unwrapped box indices (the tile's), cidx: the grid's
        auto scatter = [&](const int *uidx, const int *cidx, int f, T v) {
            const int off = tile.node_offset(uidx);
            if (off >= 0) {
                lds_add(&tmem[f * tile.plane + off], v);
                return;
            }
            long long o = I.node_off;
            for (int a = 0; a < D; ++a) o += (long long)cidx[a] * I.stride[a];
            atomicAdd(&mu[o * PS + f], v);
        };
        double gth[kThetaSlots];
        for (int kk = 0; kk < kThetaSlots; ++kk) gth[kk] = 0.0;
        const bool valid = (int)threadIdx.x < it.count;
        const int node = valid ? nodes[it.first + threadIdx.x] : 0;
        const T Lm = valid ? lam[I.node_off + node] : T(0);
        if (valid && Lm != T(0)) {
            int idx[3];
            split_node<D>(I, node, idx);
            const double *tf = time_factors(P, n, it.inst);
            double c[3];
            node_centre<D>(I, coords, tf, trig, idx, P.dt, c);
            T V[D][L], Sv[D][L], dV[D][L], dS[D][L], aV[D][L], aS[D][L];
            int o[3];
            T m[3];
            bool ok = true;
#pragma unroll
            for (int a = 0; a < D; ++a)
                ok = axis_vectors<T, QS, L, AFF, true>(I, coords, ga, w1, a, c[a], o[a], m[a],
                                                       V[a], Sv[a], dV[a], dS[a], aV[a], aS[a]) && ok;
            if (!ok) atomicOr(P.flags, 2);
            T Gz[3] = {T(0), T(0), T(0)}, Hz[3] = {T(0), T(0), T(0)};
            if constexpr (D == 1) {
#pragma unroll
                for (int i = 0; i < L; ++i) {
                    const int ci = wrap_index(o[0] + i, I.n[0], I.periodic[0]);
                    const R r = rec[I.node_off + ci];
                    Gz[0] += dV[0][i] * r.x + dS[0][i] * r.y;
                    Hz[0] += aV[0][i] * r.x + aS[0][i] * r.y;
                    int cidx[1] = {ci}, uidx[1] = {o[0] + i};
                    scatter(uidx, cidx, 0, Lm * V[0][i]);
                    scatter(uidx, cidx, 1, Lm * Sv[0][i]);
                }
            } else if constexpr (D == 2) {
#pragma unroll
                for (int i = 0; i < L; ++i) {
                    const int ci = wrap_index(o[0] + i, I.n[0], I.periodic[0]);
#pragma unroll
                    for (int j = 0; j < L; ++j) {
                        const int cj = wrap_index(o[1] + j, I.n[1], I.periodic[1]);
                        const R r = rec[I.node_off + (long long)ci * I.stride[0] + cj];
                        Gz[0] += dV[0][i] * (V[1][j] * r.x + Sv[1][j] * r.z) + dS[0][i] * V[1][j] * r.y;
                        Gz[1] += V[0][i] * (dV[1][j] * r.x + dS[1][j] * r.z) + Sv[0][i] * dV[1][j] * r.y;
                        Hz[0] += aV[0][i] * (V[1][j] * r.x + Sv[1][j] * r.z) + aS[0][i] * V[1][j] * r.y;
                        Hz[1] += V[0][i] * (aV[1][j] * r.x + aS[1][j] * r.z) + Sv[0][i] * aV[1][j] * r.y;
                        int cidx[2] = {ci, cj}, uidx[2] = {o[0] + i, o[1] + j};
                        scatter(uidx, cidx, 0, Lm * V[0][i] * V[1][j]);
                        scatter(uidx, cidx, 1, Lm * Sv[0][i] * V[1][j]);
                        scatter(uidx, cidx, 2, Lm * V[0][i] * Sv[1][j]);
                    }
                }
            } else {
                // theta-gradient first, contracting along the innermost axis: per
                // box row (i, j) twelve sums of the records against the axis-2
                // vectors, then the axis-0 and axis-1 factors once per row
                int ck[L];
#pragma unroll
                for (int kk = 0; kk < L; ++kk) ck[kk] = wrap_index(o[2] + kk, I.n[2], I.periodic[2]);
#pragma unroll
                for (int i = 0; i < L; ++i) {
                    const int ci = wrap_index(o[0] + i, I.n[0], I.periodic[0]);
#pragma unroll
                    for (int j = 0; j < L; ++j) {
                        const int cj = wrap_index(o[1] + j, I.n[1], I.periodic[1]);
                        const R *rr = rec + I.node_off + (long long)ci * I.stride[0] +
                                      (long long)cj * I.stride[1];
                        T uV = T(0), udV = T(0), uaV = T(0), g0V = T(0), g0dV = T(0), g0aV = T(0);
                        T g1V = T(0), g1dV = T(0), g1aV = T(0), g2S = T(0), g2dS = T(0), g2aS = T(0);
#pragma unroll
                        for (int kk = 0; kk < L; ++kk) {
                            const R r = rr[ck[kk]];
                            uV += V[2][kk] * r.x;
                            udV += dV[2][kk] * r.x;
                            uaV += aV[2][kk] * r.x;
                            g0V += V[2][kk] * r.y;
                            g0dV += dV[2][kk] * r.y;
                            g0aV += aV[2][kk] * r.y;
                            g1V += V[2][kk] * r.z;
                            g1dV += dV[2][kk] * r.z;
                            g1aV += aV[2][kk] * r.z;
                            g2S += Sv[2][kk] * r.w;
                            g2dS += dS[2][kk] * r.w;
                            g2aS += aS[2][kk] * r.w;
                        }
                        // d/dz_a of (V0 V1 V2 u + S0 V1 V2 g0 + V0 S1 V2 g1 + V0 V1 S2 g2)
                        const T in0 = V[1][j] * (uV + g2S) + Sv[1][j] * g1V, s0 = V[1][j] * g0V;
                        Gz[0] += dV[0][i] * in0 + dS[0][i] * s0;
                        Hz[0] += aV[0][i] * in0 + aS[0][i] * s0;
                        const T in1 = V[0][i] * (uV + g2S) + Sv[0][i] * g0V, s1 = V[0][i] * g1V;
                        Gz[1] += dV[1][j] * in1 + dS[1][j] * s1;
                        Hz[1] += aV[1][j] * in1 + aS[1][j] * s1;
                        const T v01 = V[0][i] * V[1][j], s0v1 = Sv[0][i] * V[1][j], v0s1 = V[0][i] * Sv[1][j];
                        Gz[2] += v01 * (udV + g2dS) + s0v1 * g0dV + v0s1 * g1dV;
                        Hz[2] += v01 * (uaV + g2aS) + s0v1 * g0aV + v0s1 * g1aV;
                    }
                }
                // transposed weights of box node (i, j, k): row factors
                // Lm (V0 V1, S0 V1, V0 S1) times V2, and Lm V0 V1 times S2
                const int b0 = o[0] - tile.lo[0], b1 = o[1] - tile.lo[1], b2 = o[2] - tile.lo[2];
                if (tile.use && b0 >= 0 && b0 + L <= tile.ext[0] && b1 >= 0 && b1 + L <= tile.ext[1] &&
                    b2 >= 0 && b2 + L <= tile.pitch) {
#pragma unroll
                    for (int i = 0; i < L; ++i)
#pragma unroll
                        for (int j = 0; j < L; ++j) {
                            const T fa = Lm * V[0][i] * V[1][j], fb = Lm * Sv[0][i] * V[1][j];
                            const T fc = Lm * V[0][i] * Sv[1][j];
                            double *t = tmem + ((b0 + i) * tile.ext[1] + (b1 + j)) * tile.pitch + b2;
#pragma unroll
                            for (int kk = 0; kk < L; ++kk) {
                                lds_add(t + kk, fa * V[2][kk]);
                                lds_add(t + tile.plane + kk, fb * V[2][kk]);
                                lds_add(t + 2 * tile.plane + kk, fc * V[2][kk]);
                                lds_add(t + 3 * tile.plane + kk, fa * Sv[2][kk]);
                            }
                        }
                } else {
                    for (int i = 0; i < L; ++i)
                        for (int j = 0; j < L; ++j)
                            for (int kk = 0; kk < L; ++kk) {
                                T v0 = T(0), s0 = T(0), v1 = T(0), s1 = T(0), v2 = T(0), s2 = T(0);
#pragma unroll
                                for (int t = 0; t < L; ++t) {
                                    if (t == i) { v0 = V[0][t]; s0 = Sv[0][t]; }
                                    if (t == j) { v1 = V[1][t]; s1 = Sv[1][t]; }
                                    if (t == kk) { v2 = V[2][t]; s2 = Sv[2][t]; }
                                }
                                const int cidx[3] = {wrap_index(o[0] + i, I.n[0], I.periodic[0]),
                                                     wrap_index(o[1] + j, I.n[1], I.periodic[1]),
                                                     wrap_index(o[2] + kk, I.n[2], I.periodic[2])};
                                const int uidx[3] = {o[0] + i, o[1] + j, o[2] + kk};
                                const T fa = Lm * v0 * v1;
                                scatter(uidx, cidx, 0, fa * v2);
                                scatter(uidx, cidx, 1, Lm * s0 * v1 * v2);
                                scatter(uidx, cidx, 2, Lm * v0 * s1 * v2);
                                scatter(uidx, cidx, 3, fa * s2);
                            }
                }
            }
            node_theta<D, T>(P, I, tf, trig, idx, Lm, Gz, Hz, gth);
        }
        __syncthreads();
        tile.template flush<PS>(I, mu, (T *)P.adj.stage);
        reduce_theta(red, gth, grad, it.inst);
        __syncthreads();
    }
}

// lam^{n+1} += J_F(u)^T mu_g (scatter over each node's slope stencil);
// lam_next must hold mu_u on entry.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_adjoint_slopes_T(PlanDev P, const T *__restrict__ u,
                                                             T *__restrict__ mu,
                                                             T *__restrict__ lam_next,
                                                             const WorkItem *__restrict__ items,
                                                             int first, int n_items)
{
    constexpr int PS = RecStride<D>::value;
    const WorkRange wr = work_range(first, n_items);
    for (int w = wr.begin; w < wr.end; w += wr.step) {
        const WorkItem it = items[w];
        if ((int)threadIdx.x >= it.count || it.kind != 0) continue;
        const DevInst &I = P.inst[it.inst];
        const int node = it.first + threadIdx.x;
        int idx[3];
        split_node<D>(I, node, idx);
        const T *ui = u + I.node_off;
        T *li = lam_next + I.node_off;
        for (int a = 0; a < D; ++a) {
            T *mp = &mu[(I.node_off + node) * PS + 1 + a];
            const T m = *mp;
            if (m == T(0)) continue;
            *mp = T(0);   // mu is clear again for the next step
            const int na = I.n[a];
            const double *x = P.coords + I.coord_off[a];
            const int i = idx[a];
            int il, ic, ir;
            double hl, hr;
            if (I.periodic[a]) {
                ic = (i == na - 1) ? 0 : i;
                il = (ic == 0) ? na - 2 : ic - 1;
                ir = ic + 1;
                hl = (ic == 0) ? x[na - 1] - x[na - 2] : x[ic] - x[ic - 1];
                hr = x[ic + 1] - x[ic];
            } else if (i == 0) {
                il = 0; ic = 1; ir = 2;
                hl = x[1] - x[0]; hr = x[2] - x[1];
            } else if (i == na - 1) {
                il = na - 3; ic = na - 2; ir = na - 1;
                hl = x[na - 2] - x[na - 3]; hr = x[na - 1] - x[na - 2];
            } else {
                il = i - 1; ic = i; ir = i + 1;
                hl = x[i] - x[i - 1]; hr = x[i + 1] - x[i];
            }
            const long long base = node - (long long)i * I.stride[a];
            const long long nl = base + (long long)il * I.stride[a];
            const long long nc = base + (long long)ic * I.stride[a];
            const long long nr = base + (long long)ir * I.stride[a];
            // derivative 0 where a divided difference vanishes, including
            // differences that are rounding noise of a flat stretch (below
            // 2^-30 of the values; in FP32 that is exact equality)
            const T tau = T(0x1p-30);
            const T vl = ui[nl], vc = ui[nc], vr = ui[nr];
            if (fabs(vc - vl) <= tau * (fabs(vc) + fabs(vl)) ||
                fabs(vr - vc) <= tau * (fabs(vr) + fabs(vc)))
                continue;
            const T dl = (vc - vl) / (T)hl;
            const T dr = (vr - vc) / (T)hr;
            if (!(dl * dr > T(0))) continue;
            const T den = (dl + dr) * (dl + dr);
            const T gdl = T(2) * dr * dr / den;
            const T gdr = T(2) * dl * dl / den;
            atomicAdd(&li[nl], m * (-gdl / (T)hl));
            atomicAdd(&li[nc], m * (gdl / (T)hl - gdr / (T)hr));
            atomicAdd(&li[nr], m * (gdr / (T)hr));
        }
    }
}

// lam <- mu_u (field 0 of the records) over the nodes of a work list (node
// runs), clearing mu_u for the next step.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_mu_value(PlanDev P, T *__restrict__ mu,
                                                     T *__restrict__ lam,
                                                     const WorkItem *__restrict__ items,
                                                     int first, int n_items)
{
    constexpr int PS = RecStride<D>::value;
    const WorkRange wr = work_range(first, n_items);
    for (int w = wr.begin; w < wr.end; w += wr.step) {
        const WorkItem it = items[w];
        if ((int)threadIdx.x >= it.count || it.kind != 0) continue;
        const long long g = P.inst[it.inst].node_off + it.first + threadIdx.x;
        lam[g] = mu[g * PS];
        mu[g * PS] = T(0);
    }
}

// Exit nodes carry no sensitivity; a periodic image passes its cotangent to
// the node it copies.  cls: 0 active, 1 exit, 2 image of an active node,
// 3 image of an exit node.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_fold_images(PlanDev P, T *__restrict__ lam,
                                                        const WorkItem *__restrict__ items,
                                                        int first, int n_items)
{
    const WorkRange wr = work_range(first, n_items);
    for (int w = wr.begin; w < wr.end; w += wr.step) {
        const WorkItem it = items[w];
        if ((int)threadIdx.x >= it.count || it.kind != 0) continue;
        const DevInst &I = P.inst[it.inst];
        const int node = it.first + threadIdx.x;
        const long long g = I.node_off + node;
        const unsigned char c = P.chi[g];
        if (c == 0) continue;
        if (c == 2) {
            int idx[3];
            split_node<D>(I, node, idx);
            long long rep = node;
            for (int a = 0; a < D; ++a)
                if (I.periodic[a] && idx[a] == I.n[a] - 1)
                    rep -= (long long)(I.n[a] - 1) * I.stride[a];
            atomicAdd(&lam[I.node_off + rep], lam[g]);
        }
        lam[g] = T(0);
    }
}

// ---------------------------------------------------------------------------
// Fields of an FP64 sub-plan in the layout (and precision) of its FP32 parent
// plan.  items: every node of every instance (node runs).
// ---------------------------------------------------------------------------
template <bool OUT>
__global__ void __launch_bounds__(kBlock) k_convert(PlanDev P, const WorkItem *__restrict__ items,
                                                    int n_items, double *__restrict__ u,
                                                    float *__restrict__ f)
{
    const WorkRange wr = work_range(0, n_items);
    for (int w = wr.begin; w < wr.end; w += wr.step) {
        const WorkItem it = items[w];
        if ((int)threadIdx.x >= it.count) continue;
        const DevInst &I = P.inst[it.inst];
        const long long j = it.first + threadIdx.x;
        if (OUT) f[I.out_off + j] = (float)u[I.node_off + j];
        else u[I.node_off + j] = (double)f[I.out_off + j];
    }
}

// Largest |a - b| over each instance's nodes (a wave-level maximum, then one
// atomic per wave on the bit pattern, which orders like the value for
// non-negative doubles; a NaN compares above every number).
__global__ void __launch_bounds__(kBlock) k_inst_maxdiff(PlanDev P, const WorkItem *__restrict__ items,
                                                         int n_items, const double *__restrict__ a,
                                                         const float *__restrict__ b,
                                                         unsigned long long *__restrict__ out)
{
    const WorkRange wr = work_range(0, n_items);
    for (int w = wr.begin; w < wr.end; w += wr.step) {
        const WorkItem it = items[w];
        const DevInst &I = P.inst[it.inst];
        double v = 0.0;
        if ((int)threadIdx.x < it.count) {
            const long long j = I.node_off + it.first + threadIdx.x;
            v = fabs(a[j] - (double)b[j]);
            if (v != v) v = __longlong_as_double(0x7ff8000000000000LL);
        }
        unsigned long long bits = (unsigned long long)__double_as_longlong(v);
        for (int off = 32; off > 0; off >>= 1) {
            const unsigned long long o = __shfl_xor(bits, off, 64);
            bits = o > bits ? o : bits;
        }
        if ((threadIdx.x % 64) == 0 && bits) atomicMax(&out[it.inst], bits);
    }
}

// ---------------------------------------------------------------------------
// Step-operator hooks: A_n = Q Psi^n of Eq. (e36) as a linear map from the
// (d + 1) fields [u; g_0; ..; g_{d-1}] (values and nodal slopes, the column
// blocks of Psi^n) to the active rows, applied to caller data instead of the
// slope pass' records.
// ---------------------------------------------------------------------------

// fields x[f * n + i] (f = 0 value, 1 + a slope along axis a) -> records
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_pack_fields(long long n, const T *__restrict__ x,
                                                        T *__restrict__ packed)
{
    constexpr int PS = RecStride<D>::value;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
#pragma unroll
        for (int f = 0; f < PS; ++f) packed[i * PS + f] = (f <= D) ? x[f * n + i] : T(0);
}

// records -> fields (inverse of k_pack_fields)
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_unpack_fields(long long n, const T *__restrict__ rec,
                                                          T *__restrict__ x)
{
    constexpr int PS = RecStride<D>::value;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
#pragma unroll
        for (int f = 0; f <= D; ++f) x[f * n + i] = rec[i * PS + f];
}

// out = a - b (b may be null: out = a) on active nodes, 0 on all others
template <typename T>
__global__ void __launch_bounds__(kBlock) k_masked_diff(const unsigned char *__restrict__ cls,
                                                        long long n, const T *a, const T *b,
                                                        T *out)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        out[i] = (cls[i] == 0) ? (b ? a[i] - b[i] : a[i]) : T(0);
}

}  // namespace

// ---------------------------------------------------------------------------
// Launch helpers
// ---------------------------------------------------------------------------

#define FK_DISPATCH_G(G_, ...)                                   \
    switch (G_) {                                                \
    case 1: { constexpr int G = 1; __VA_ARGS__; } break;         \
    case 2: { constexpr int G = 2; __VA_ARGS__; } break;         \
    case 4: { constexpr int G = 4; __VA_ARGS__; } break;         \
    case 8: { constexpr int G = 8; __VA_ARGS__; } break;         \
    case 16: { constexpr int G = 16; __VA_ARGS__; } break;       \
    case 32: { constexpr int G = 32; __VA_ARGS__; } break;       \
    case 64: { constexpr int G = 64; __VA_ARGS__; } break;       \
    default: return hipErrorInvalidValue;                        \
    }

#define FK_DISPATCH_D(D_, ...)                                   \
    switch (D_) {                                                \
    case 1: { constexpr int D = 1; __VA_ARGS__; } break;         \
    case 2: { constexpr int D = 2; __VA_ARGS__; } break;         \
    case 3: { constexpr int D = 3; __VA_ARGS__; } break;         \
    default: return hipErrorInvalidValue;                        \
    }

static inline int flat_grid(long long n)
{
    long long g = (n + kBlock - 1) / kBlock;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace fk
