/*
 * fkoracle.c -- CPU reference ("oracle") of the backward Feynman-Kac scheme for
 * the exit-time probability (Yang, Zhang, del-Castillo-Negrete, Stoyanov,
 * "A Feynman-Kac based numerical method for the exit time probability of a
 * class of transport problems").
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code with
 * the GPU library.  Everything is plain FP64 C99, written for a reader to check
 * against the paper by eye: no blocking, fusion or reordering beyond what the
 * scheme states.  OpenMP only splits the loop over grid nodes.
 *
 * What it computes (paper Section 3.1, Scheme 1; matrix form Eq. (e36)):
 *   u^N = chi (1 on exit nodes, 0 elsewhere);
 *   for n = N-1 .. 0, for every active node x_j:
 *     z_jq = x_j + b(t_n, x_j) dt + sigma sqrt(2 dt) a_q          (Eq. (e31))
 *     u^n_j = sum_q w_q * (z_jq in exit region ? 1 : I[u^{n+1}](z_jq))
 *                                                         (Eq. (quad), (e304))
 *   where I is the cubic Hermite interpolant with PCHIP slopes (Eq. (Lag11),
 *   the 1D Hermite form of Section 3.1.2 and Eq. (e300)), taken as a tensor
 *   product over axes with value and first-derivative basis functions only.
 *
 * Build: gcc -O2 -std=c99 -fopenmp -ffp-contract=off -fPIC -shared
 *
 * Evaluation order of the landing point (kept identical in every
 * implementation so that landing cells agree bit for bit): sq = sqrt(2 dt);
 * S = sqrt(2 D) * sq; c_i = x_i + b_i * dt; z_i = c_i + S * a_{q_i}; each
 * product rounded separately (no fused multiply-add).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define FKO_COEF_CONST 0
#define FKO_COEF_CELLULAR2D 1
#define FKO_COEF_ABC3D 2
#define FKO_COEF_ROLLS2D 3
#define FKO_COEF_RUNAWAY3D 4
#define FKO_FACE_EXIT1 0        /* a point on or beyond the face exits, value 1 */
#define FKO_FACE_EXIT0 1        /* it exits with value 0 */
#define FKO_FACE_REFLECT 2      /* it is reflected back into the domain */
#define FKO_REGION_BOX 0
#define FKO_REGION_BALL 1

typedef struct {
    int d;                  /* space dimension, 1..3 */
    int n[3];               /* nodes per axis */
    const double *x[3];     /* node coordinates per axis, increasing */
    int periodic[3];        /* node n-1 is the image of node 0 */
    int coef_kind;          /* FKO_COEF_* */
    double p[16];           /* drift (and, for the runaway model, diffusion) parameters */
    double D;               /* diffusion: sigma = sqrt(2 D) I */
    int region_kind;        /* FKO_REGION_* */
    double c[3];            /* ball centre */
    double r;               /* ball radius */
    int gh_n;               /* Q*: nodes of the 1D Gauss-Hermite rule */
    const double *gh_a;     /* 1D nodes */
    const double *gh_w;     /* 1D weights (sum 1) */
    double dt;
    int n_steps;
    double t0;              /* step n evaluates coefficients at t0 + n dt */
    int hermite;            /* 1: values and first derivatives (R1); 2: with the
                               mixed derivatives (twist fields, R2) */
    int face[3][2];         /* per non-periodic axis, low and high face: FKO_FACE_* */
} fko_problem;

/* ------------------------------------------------------------------------ */
/* Grid bookkeeping                                                          */
/* ------------------------------------------------------------------------ */

long fko_num_nodes(const fko_problem *P)
{
    long J = 1;
    for (int a = 0; a < P->d; a++) J *= P->n[a];
    return J;
}

static void node_index(const fko_problem *P, long j, int *i)
{
    for (int a = P->d - 1; a >= 0; a--) {
        i[a] = (int)(j % P->n[a]);
        j /= P->n[a];
    }
}

static long node_linear(const fko_problem *P, const int *i)
{
    long j = 0;
    for (int a = 0; a < P->d; a++) j = j * P->n[a] + i[a];
    return j;
}

/* Exit test for a point (the paper's domain D is an open box, Section 2;
 * points on or beyond a non-periodic face have exited.  For a ball target the
 * exit region also holds every point with |z - c| >= r).  Returns -1 if z
 * does not exit, else the value it takes: 1 through an FKO_FACE_EXIT1 face or
 * the ball, 0 through an FKO_FACE_EXIT0 face (the face of the lowest axis
 * decides, low face before high face); reflecting faces never exit. */
int fko_exit_value(const fko_problem *P, const double *z)
{
    for (int a = 0; a < P->d; a++) {
        if (P->periodic[a]) continue;
        if (P->face[a][0] != FKO_FACE_REFLECT && z[a] <= P->x[a][0])
            return P->face[a][0] == FKO_FACE_EXIT0 ? 0 : 1;
        if (P->face[a][1] != FKO_FACE_REFLECT && z[a] >= P->x[a][P->n[a] - 1])
            return P->face[a][1] == FKO_FACE_EXIT0 ? 0 : 1;
    }
    if (P->region_kind == FKO_REGION_BALL) {
        double s = 0.0;
        for (int a = 0; a < P->d; a++) {
            double t = z[a] - P->c[a];
            s = s + t * t;
        }
        if (s >= P->r * P->r) return 1;
    }
    return -1;
}

int fko_is_exit_point(const fko_problem *P, const double *z)
{
    return fko_exit_value(P, z) >= 0;
}

/* 0 = active node, 1 = exit node (u = 1 for all n, terminal value chi = 1),
 * 2 = periodic image of another node (takes that node's value). */
int fko_node_class(const fko_problem *P, long j)
{
    int i[3];
    double x[3];
    node_index(P, j, i);
    for (int a = 0; a < P->d; a++)
        if (P->periodic[a] && i[a] == P->n[a] - 1) return 2;
    for (int a = 0; a < P->d; a++) x[a] = P->x[a][i[a]];
    return fko_is_exit_point(P, x) ? 1 : 0;
}

static long representative(const fko_problem *P, long j)
{
    int i[3];
    node_index(P, j, i);
    for (int a = 0; a < P->d; a++)
        if (P->periodic[a] && i[a] == P->n[a] - 1) i[a] = 0;
    return node_linear(P, i);
}

/* Sorted list of active nodes; returns the count. */
long fko_active_nodes(const fko_problem *P, long *out)
{
    long J = fko_num_nodes(P), m = 0;
    for (long j = 0; j < J; j++)
        if (fko_node_class(P, j) == 0) {
            if (out) out[m] = j;
            m++;
        }
    return m;
}

/* ------------------------------------------------------------------------ */
/* Coefficients b(t, x), sigma (paper Eq. (e1)); sigma = sqrt(2 D) I         */
/* except for the runaway-electron model of Section 4.3                      */
/* ------------------------------------------------------------------------ */

/* Runaway-electron model (Section 4.3, Eq. (ex32d)): state (p, xi, r),
 * parameters p[] = (E, tau, Z, delta, nu_ee, v_T, r_D, W, Delta_p, V_0, D_0,
 * t_*, That_0, That_f, Ttilde, m c^2).  With t_* > 0 the electric field and
 * the collision parameters follow the thermal-quench model of Section 4.3:
 * That(t) = That_f + (That_0 - That_f) exp(-t / t_*), v_T = sqrt(That /
 * Ttilde), nu_ee = (Ttilde / That)^(3/2) lnLambda(That) / lnLambda(Ttilde),
 * lnLambda(T) = 14.9 - ln(0.28) / 2 + ln T, delta = sqrt(2 That / m c^2),
 * E = E_0 (That_0 / That)^(3/2) (p[0] is then E_0). */
typedef struct { double E, nu, vT, delta; } re_params;

static re_params re_at(const fko_problem *P, double t)
{
    const double *p = P->p;
    re_params q;
    if (p[11] > 0.0) {
        double Th = p[13] + (p[12] - p[13]) * exp(-t / p[11]);
        double lnh = 14.9 - 0.5 * log(0.28) + log(Th);
        double lnt = 14.9 - 0.5 * log(0.28) + log(p[14]);
        q.vT = sqrt(Th / p[14]);
        q.nu = pow(p[14] / Th, 1.5) * lnh / lnt;
        q.delta = sqrt(2.0 * Th / p[15]);
        q.E = p[0] * pow(p[12] / Th, 1.5);
    } else {
        q.E = p[0]; q.delta = p[3]; q.nu = p[4]; q.vT = p[5];
    }
    return q;
}

/* Collision functions at momentum pm (Section 4.3): phi(y) = erf(y),
 * psi(y) = (phi - y phi') / (2 y^2), y = p / gamma, gamma = sqrt(1 +
 * (delta p)^2); C_A = nu v_T^2 psi / y, C_B = nu v_T^2 (Z + phi - psi +
 * y^2 delta^4 / 2) / (2 y), C_F = 2 nu v_T psi, and dC_A/dp (psi' =
 * phi' - 2 psi / y, dy/dp = gamma^-3).  out = (C_A, C_B, C_F, dC_A/dp). */
static void re_collisions(const fko_problem *P, const re_params *q, double pm, double *out)
{
    double Z = P->p[2];
    double gam = sqrt(1.0 + (q->delta * pm) * (q->delta * pm));
    double y = pm / gam;
    double phi = erf(y);
    double dphi = 2.0 / sqrt(M_PI) * exp(-y * y);
    double psi = (phi - y * dphi) / (2.0 * y * y);
    double dpsi = dphi - 2.0 * psi / y;
    double k2 = q->nu * q->vT * q->vT;
    out[0] = k2 * psi / y;
    out[1] = 0.5 * k2 / y * (Z + phi - psi + 0.5 * y * y * pow(q->delta, 4));
    out[2] = 2.0 * q->nu * q->vT * psi;
    out[3] = k2 * (dpsi * y - psi) / (y * y) / (gam * gam * gam);
}

void fko_re_coeffs(const fko_problem *P, double t, double pm, double *out)
{
    re_params q = re_at(P, t);
    re_collisions(P, &q, pm, out);
}

/* Radial diffusivity D(r, p) = D_0 / 2 (1 + tanh((r - r_D) / W)) exp(-(p /
 * Delta_p)^2) and its r-derivative. */
static void re_radial(const fko_problem *P, double pm, double r, double *D, double *dD)
{
    const double *p = P->p;
    double th = tanh((r - p[6]) / p[7]);
    double e = exp(-(pm / p[8]) * (pm / p[8]));
    *D = 0.5 * p[10] * (1.0 + th) * e;
    *dD = 0.5 * p[10] * (1.0 - th * th) / p[7] * e;
}

/* Diffusion coefficient of each axis at (t, x): sigma_a (the SDE's dW
 * factor; sigma = sqrt(2 D) for the other models). */
void fko_sigma(const fko_problem *P, double t, const double *x, double *sig)
{
    if (P->coef_kind == FKO_COEF_RUNAWAY3D) {
        re_params q = re_at(P, t);
        double c[4], D, dD;
        re_collisions(P, &q, x[0], c);
        re_radial(P, x[0], x[2], &D, &dD);
        double om = 1.0 - x[1] * x[1];
        sig[0] = sqrt(2.0 * c[0]);
        sig[1] = sqrt(2.0 * c[1]) / x[0] * sqrt(om > 0.0 ? om : 0.0);
        sig[2] = sqrt(2.0 * D);
        return;
    }
    double s = sqrt(2.0 * P->D);
    for (int a = 0; a < P->d; a++) sig[a] = s;
}

void fko_drift(const fko_problem *P, double t, const double *x, double *b)
{
    const double *p = P->p;
    if (P->coef_kind == FKO_COEF_CONST) {
        for (int a = 0; a < P->d; a++) b[a] = p[a];
    } else if (P->coef_kind == FKO_COEF_CELLULAR2D) {
        /* psi = A sin(pi (x + eps sin(omega t))) sin(pi y);
         * b = (-d psi/dy, d psi/dx). */
        double ph = p[1] * sin(p[2] * t);
        double arg = M_PI * (x[0] + ph);
        double sa = sin(arg), ca = cos(arg);
        double sy = sin(M_PI * x[1]), cy = cos(M_PI * x[1]);
        double Api = p[0] * M_PI;
        b[0] = -(Api * sa * cy);
        b[1] = Api * ca * sy;
    } else if (P->coef_kind == FKO_COEF_RUNAWAY3D) {
        /* Eq. (ex32d): the p drift includes (1/p^2) d/dp (p^2 C_A) =
         * 2 C_A / p + dC_A/dp; the r drift V(r) + dD/dr with
         * V = V_0 [r > r_D] */
        re_params q = re_at(P, t);
        double c[4], D, dD;
        double pm = x[0], xi = x[1], r = x[2];
        double gam = sqrt(1.0 + (q.delta * pm) * (q.delta * pm));
        double om = 1.0 - xi * xi;
        re_collisions(P, &q, pm, c);
        re_radial(P, pm, r, &D, &dD);
        b[0] = q.E * xi - gam * pm / p[1] * om - c[2] + 2.0 * c[0] / pm + c[3];
        b[1] = q.E * om / pm - xi * om / (p[1] * gam) - 2.0 * xi * c[1] / (pm * pm);
        b[2] = (r > p[6] ? p[9] : 0.0) + dD;
    } else if (P->coef_kind == FKO_COEF_ROLLS2D) {
        /* Section 4.2: Pe v with v_1 = -pi cos(pi x_2) [sin(n x_1) + eps f(t) cos(n x_1)],
         * v_2 = n sin(pi x_2) [cos(n x_1) - eps f(t) sin(n x_1)], f(t) = cos(omega t);
         * p = (Pe, eps, omega, n). */
        double e = p[1] * cos(p[2] * t);
        double s1 = sin(p[3] * x[0]), c1 = cos(p[3] * x[0]);
        double s2 = sin(M_PI * x[1]), c2 = cos(M_PI * x[1]);
        b[0] = -(p[0] * M_PI * c2 * (s1 + e * c1));
        b[1] = p[0] * p[3] * s2 * (c1 - e * s1);
    } else {
        /* ABC flow, amplitudes modulated by f(t) = 1 + amp sin t */
        double f = 1.0 + p[3] * sin(t);
        double Af = p[0] * f, Bf = p[1] * f, Cf = p[2] * f;
        b[0] = Af * sin(x[2]) + Cf * cos(x[1]);
        b[1] = Bf * sin(x[0]) + Af * cos(x[2]);
        b[2] = Cf * sin(x[1]) + Bf * cos(x[0]);
    }
}

/* Number of differentiable parameters theta = (drift parameters..., D). */
int fko_num_theta(const fko_problem *P)
{
    if (P->coef_kind == FKO_COEF_CONST) return P->d + 1;
    if (P->coef_kind == FKO_COEF_CELLULAR2D) return 4;
    if (P->coef_kind == FKO_COEF_ROLLS2D) return 4;   /* (Pe, eps, omega, D); n is a count */
    if (P->coef_kind == FKO_COEF_RUNAWAY3D) return 1; /* no adjoint for this model */
    return 5;
}

/* d z_i / d theta_k for one landing point; dz[k * 3 + i].  a[i] is the GH
 * node used on axis i. */
static void dz_dtheta(const fko_problem *P, double t, const double *x,
                      const double *a, double *dz)
{
    const double *p = P->p;
    int nt = fko_num_theta(P);
    double dt = P->dt;
    for (int k = 0; k < nt * 3; k++) dz[k] = 0.0;
    if (P->coef_kind == FKO_COEF_CONST) {
        for (int i = 0; i < P->d; i++) dz[i * 3 + i] = dt;
    } else if (P->coef_kind == FKO_COEF_CELLULAR2D) {
        double A = p[0], eps = p[1], om = p[2];
        double ph = eps * sin(om * t);
        double phi = M_PI * (x[0] + ph);
        double sphi = sin(phi), cphi = cos(phi);
        double sy = sin(M_PI * x[1]), cy = cos(M_PI * x[1]);
        /* d b / d A */
        dz[0 * 3 + 0] = dt * (-M_PI * sphi * cy);
        dz[0 * 3 + 1] = dt * (M_PI * cphi * sy);
        /* d b / d phi, chained with d phi / d eps and d phi / d omega */
        double db0 = -A * M_PI * cphi * cy;
        double db1 = -A * M_PI * sphi * sy;
        double dphi_deps = M_PI * sin(om * t);
        double dphi_dom = M_PI * eps * t * cos(om * t);
        dz[1 * 3 + 0] = dt * db0 * dphi_deps;
        dz[1 * 3 + 1] = dt * db1 * dphi_deps;
        dz[2 * 3 + 0] = dt * db0 * dphi_dom;
        dz[2 * 3 + 1] = dt * db1 * dphi_dom;
    } else if (P->coef_kind == FKO_COEF_ROLLS2D) {
        double Pe = p[0], eps = p[1], om = p[2], nn = p[3];
        double e = eps * cos(om * t);
        double s1 = sin(nn * x[0]), c1 = cos(nn * x[0]);
        double s2 = sin(M_PI * x[1]), c2 = cos(M_PI * x[1]);
        /* d b / d Pe = v */
        dz[0 * 3 + 0] = dt * (-(M_PI * c2 * (s1 + e * c1)));
        dz[0 * 3 + 1] = dt * (nn * s2 * (c1 - e * s1));
        /* d b / d e, chained with d e / d eps = cos(omega t) and
         * d e / d omega = -eps t sin(omega t) */
        double db0 = -(Pe * M_PI * c2 * c1);
        double db1 = -(Pe * nn * s2 * s1);
        double de_deps = cos(om * t);
        double de_dom = -(eps * t * sin(om * t));
        dz[1 * 3 + 0] = dt * db0 * de_deps;
        dz[1 * 3 + 1] = dt * db1 * de_deps;
        dz[2 * 3 + 0] = dt * db0 * de_dom;
        dz[2 * 3 + 1] = dt * db1 * de_dom;
    } else {
        double A = p[0], B = p[1], C = p[2], amp = p[3];
        double st = sin(t), f = 1.0 + amp * st;
        double sx = sin(x[0]), cx = cos(x[0]), sy = sin(x[1]), cy = cos(x[1]);
        double sz = sin(x[2]), cz = cos(x[2]);
        dz[0 * 3 + 0] = dt * f * sz;   /* A */
        dz[0 * 3 + 1] = dt * f * cz;
        dz[1 * 3 + 1] = dt * f * sx;   /* B */
        dz[1 * 3 + 2] = dt * f * cx;
        dz[2 * 3 + 0] = dt * f * cy;   /* C */
        dz[2 * 3 + 2] = dt * f * sy;
        dz[3 * 3 + 0] = dt * st * (A * sz + C * cy);   /* amp */
        dz[3 * 3 + 1] = dt * st * (B * sx + A * cz);
        dz[3 * 3 + 2] = dt * st * (C * sy + B * cx);
    }
    /* D enters through S = sqrt(2 D) sqrt(2 dt): dS/dD = S / (2 D) */
    double S = sqrt(2.0 * P->D) * sqrt(2.0 * P->dt);
    for (int i = 0; i < P->d; i++) dz[(nt - 1) * 3 + i] = a[i] * S / (2.0 * P->D);
}

/* ------------------------------------------------------------------------ */
/* Landing points (Euler step, Eq. (ref-X) with the quadrature substitution   */
/* of Eq. (expec)-(e31)).                                                    */
/* ------------------------------------------------------------------------ */

/* Tensor index q -> per-axis GH indices, last axis fastest. */
static void split_q(const fko_problem *P, int q, int *qi)
{
    for (int a = P->d - 1; a >= 0; a--) {
        qi[a] = q % P->gh_n;
        q /= P->gh_n;
    }
}

static double tensor_weight(const fko_problem *P, const int *qi)
{
    double w = P->gh_w[qi[0]];
    for (int a = 1; a < P->d; a++) w = w * P->gh_w[qi[a]];
    return w;
}

void fko_landing(const fko_problem *P, int n, long j, int q, double *z)
{
    int i[3], qi[3];
    double x[3], b[3], sig[3];
    double t = P->t0 + (double)n * P->dt;
    double sq = sqrt(2.0 * P->dt);
    node_index(P, j, i);
    for (int a = 0; a < P->d; a++) x[a] = P->x[a][i[a]];
    fko_drift(P, t, x, b);
    fko_sigma(P, t, x, sig);
    split_q(P, q, qi);
    for (int a = 0; a < P->d; a++) {
        double S = sig[a] * sq;
        double c = x[a] + b[a] * P->dt;
        z[a] = c + S * P->gh_a[qi[a]];
        const double *xa = P->x[a];
        double lo = xa[0], hi = xa[P->n[a] - 1];
        if (P->periodic[a]) {
            double L = hi - lo;
            if (z[a] >= hi) z[a] = z[a] - L;
            else if (z[a] < lo) z[a] = z[a] + L;
        } else {
            /* a reflecting face mirrors the point back into the domain */
            if (P->face[a][0] == FKO_FACE_REFLECT && z[a] < lo) z[a] = lo + (lo - z[a]);
            if (P->face[a][1] == FKO_FACE_REFLECT && z[a] > hi) z[a] = hi - (z[a] - hi);
        }
    }
}

/* Cell of z on an axis: max{k : x_k <= z}, clamped to [0, n-2]. */
int fko_cell(const double *x, int n, double z)
{
    if (z < x[0]) return 0;
    if (z >= x[n - 1]) return n - 2;
    int lo = 0, hi = n - 1;          /* x[lo] <= z < x[hi] */
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (x[mid] <= z) lo = mid;
        else hi = mid;
    }
    return lo;
}

/* ------------------------------------------------------------------------ */
/* PCHIP slopes (Eq. (e300) and the end-node rule that follows it)           */
/* ------------------------------------------------------------------------ */

/* Harmonic-mean slope of two divided differences: 0 unless they have the same
 * (nonzero) sign, else 2 / (1/a + 1/b) = 2ab / (a + b). */
static double pchip_pair(double a, double b)
{
    if (a * b > 0.0) return 2.0 * a * b / (a + b);
    return 0.0;
}

/* Per node, the slope along axis ax needs three nodes: (il, ic, ir) along the
 * line and the two spacings.  Returns the indices along the axis. */
static void slope_stencil(const fko_problem *P, int ax, int i, int *il, int *ic,
                          int *ir, double *hl, double *hr, int *kind)
{
    int n = P->n[ax];
    const double *x = P->x[ax];
    *kind = 0;  /* 0: centred (left, right); 1: first node; 2: last node */
    if (P->periodic[ax]) {
        int c = (i == n - 1) ? 0 : i;
        *ic = c;
        *il = (c == 0) ? n - 2 : c - 1;
        *ir = c + 1;
        *hl = (c == 0) ? x[n - 1] - x[n - 2] : x[c] - x[c - 1];
        *hr = x[c + 1] - x[c];
    } else if (i == 0) {
        *kind = 1;   /* uses delta_0 = (u1-u0)/h0, delta_1 = (u2-u1)/h1 */
        *il = 0; *ic = 1; *ir = 2;
        *hl = x[1] - x[0];
        *hr = x[2] - x[1];
    } else if (i == n - 1) {
        *kind = 2;   /* uses delta_{n-2} and delta_{n-3} */
        *il = n - 3; *ic = n - 2; *ir = n - 1;
        *hl = x[n - 2] - x[n - 3];
        *hr = x[n - 1] - x[n - 2];
    } else {
        *il = i - 1; *ic = i; *ir = i + 1;
        *hl = x[i] - x[i - 1];
        *hr = x[i + 1] - x[i];
    }
}

/* PCHIP slope of the field f along axis ax at every node: out[j]. */
static void slope_along(const fko_problem *P, int ax, const double *f, double *out)
{
    long J = fko_num_nodes(P);
#pragma omp parallel for schedule(static)
    for (long j = 0; j < J; j++) {
        int i[3], il, ic, ir, kind;
        double hl, hr;
        node_index(P, j, i);
        slope_stencil(P, ax, i[ax], &il, &ic, &ir, &hl, &hr, &kind);
        int t[3];
        memcpy(t, i, sizeof(t));
        t[ax] = il; double ul = f[node_linear(P, t)];
        t[ax] = ic; double uc = f[node_linear(P, t)];
        t[ax] = ir; double ur = f[node_linear(P, t)];
        double dl = (uc - ul) / hl;
        double dr = (ur - uc) / hr;
        out[j] = pchip_pair(dl, dr);
    }
}

/* Derivative fields of the interpolant.  Field f = 0 .. d-1 is the slope
 * along axis f.  With the mixed derivatives (R2) the fields that follow are
 * the twist fields, one per set S of two or more axes, in the order
 * {0,1}, {0,2}, {1,2}, {0,1,2} (2D: {0,1} only); the field of S is the PCHIP
 * slope along the largest axis of S of the field of S without that axis, i.e.
 * the one-dimensional rule composed in increasing axis order
 * (u_xy = D_y(D_x u), u_xyz = D_z(D_y(D_x u))). */
int fko_num_fields(const fko_problem *P)
{
    return P->hermite == 2 ? (1 << P->d) - 1 : P->d;
}

/* Axis set of derivative field f, as a bit mask (bit a: axis a). */
static int field_mask(const fko_problem *P, int f)
{
    static const int twist3[4] = {3, 5, 6, 7};
    if (f < P->d) return 1 << f;
    return P->d == 2 ? 3 : twist3[f - 3];
}

/* g[f * J + j] = derivative field f (fko_num_fields) at node j. */
void fko_slopes(const fko_problem *P, const double *u, double *g)
{
    long J = fko_num_nodes(P);
    for (int ax = 0; ax < P->d; ax++) slope_along(P, ax, u, g + (long)ax * J);
    for (int f = P->d; f < fko_num_fields(P); f++) {
        int m = field_mask(P, f), top = 0;
        for (int a = 0; a < P->d; a++)
            if (m & (1 << a)) top = a;
        int base = m & ~(1 << top), fb = -1;
        for (int k = 0; k < f; k++)
            if (field_mask(P, k) == base) fb = k;
        slope_along(P, top, g + (long)fb * J, g + (long)f * J);
    }
}

/* ------------------------------------------------------------------------ */
/* Cubic Hermite interpolant (Section 3.1.2), tensor product of 1D value and  */
/* slope basis functions; s in [0, 1] is the position inside the cell.       */
/* ------------------------------------------------------------------------ */

static double H0(int c, double s)   /* value basis: left (c=0) / right (c=1) */
{
    return c ? s * s * (3.0 - 2.0 * s) : (1.0 + 2.0 * s) * (1.0 - s) * (1.0 - s);
}
static double H1(int c, double s)   /* slope basis (times h) */
{
    return c ? s * s * (s - 1.0) : s * (1.0 - s) * (1.0 - s);
}
static double dH0(int c, double s)
{
    return c ? 6.0 * s - 6.0 * s * s : 6.0 * s * s - 6.0 * s;
}
static double dH1(int c, double s)
{
    return c ? 3.0 * s * s - 2.0 * s : 1.0 - 4.0 * s + 3.0 * s * s;
}

static void locate(const fko_problem *P, const double *z, int *k, double *s, double *h)
{
    for (int a = 0; a < P->d; a++) {
        const double *x = P->x[a];
        k[a] = fko_cell(x, P->n[a], z[a]);
        h[a] = x[k[a] + 1] - x[k[a]];
        s[a] = (z[a] - x[k[a]]) / h[a];
    }
}

/* Value of the full tensor cubic Hermite interpolant (R2) of u and its
 * derivative fields at z: per cell corner and per axis set S (S empty: u),
 * the field of S times prod_{a in S} h_a H1(s_a) prod_{a not in S} H0(s_a). */
static double interp_full(const fko_problem *P, const double *u, const double *g,
                          const double *z)
{
    long J = fko_num_nodes(P);
    int k[3], corner[3], bit[3];
    double s[3], h[3];
    locate(P, z, k, s, h);
    int nf = fko_num_fields(P);
    double val = 0.0;
    for (int c = 0; c < (1 << P->d); c++) {
        for (int a = 0; a < P->d; a++) {
            bit[a] = (c >> (P->d - 1 - a)) & 1;
            corner[a] = k[a] + bit[a];
        }
        long node = node_linear(P, corner);
        for (int f = -1; f < nf; f++) {
            int m = f < 0 ? 0 : field_mask(P, f);
            double w = 1.0;
            for (int a = 0; a < P->d; a++)
                w = w * ((m & (1 << a)) ? h[a] * H1(bit[a], s[a]) : H0(bit[a], s[a]));
            val += (f < 0 ? u[node] : g[(long)f * J + node]) * w;
        }
    }
    return val;
}

/* Value of the interpolant of (u, g) at z; optionally its gradient. */
static double interp(const fko_problem *P, const double *u, const double *g,
                     const double *z, double *grad)
{
    long J = fko_num_nodes(P);
    int k[3], corner[3];
    double s[3], h[3];
    if (P->hermite == 2) return interp_full(P, u, g, z);
    locate(P, z, k, s, h);
    double val = 0.0;
    if (grad) for (int a = 0; a < P->d; a++) grad[a] = 0.0;
    for (int c = 0; c < (1 << P->d); c++) {
        for (int a = 0; a < P->d; a++) corner[a] = k[a] + ((c >> (P->d - 1 - a)) & 1);
        int bit[3];
        for (int a = 0; a < P->d; a++) bit[a] = (c >> (P->d - 1 - a)) & 1;
        long node = node_linear(P, corner);
        /* value term: u * prod_a H0 */
        double wv = 1.0;
        for (int a = 0; a < P->d; a++) wv = wv * H0(bit[a], s[a]);
        val += u[node] * wv;
        /* slope terms: g_a * h_a H1(s_a) * prod_{i != a} H0(s_i) */
        for (int a = 0; a < P->d; a++) {
            double ws = h[a] * H1(bit[a], s[a]);
            for (int i = 0; i < P->d; i++)
                if (i != a) ws = ws * H0(bit[i], s[i]);
            val += g[a * J + node] * ws;
        }
        if (grad) {
            /* d/dz_m: differentiate the axis-m factor (d/dz = (1/h_m) d/ds) */
            for (int m = 0; m < P->d; m++) {
                double dv = dH0(bit[m], s[m]) / h[m];
                for (int i = 0; i < P->d; i++)
                    if (i != m) dv = dv * H0(bit[i], s[i]);
                double acc = u[node] * dv;
                for (int a = 0; a < P->d; a++) {
                    double ds;
                    if (a == m) ds = dH1(bit[a], s[a]);   /* h_a H1' / h_a */
                    else ds = h[a] * H1(bit[a], s[a]) * dH0(bit[m], s[m]) / h[m];
                    for (int i = 0; i < P->d; i++)
                        if (i != a && i != m) ds = ds * H0(bit[i], s[i]);
                    acc += g[a * J + node] * ds;
                }
                grad[m] += acc;
            }
        }
    }
    return val;
}

double fko_interp(const fko_problem *P, const double *u, const double *g, const double *z)
{
    return interp(P, u, g, z, NULL);
}

void fko_interp_grad(const fko_problem *P, const double *u, const double *g,
                     const double *z, double *grad)
{
    (void)interp(P, u, g, z, grad);
}

/* ------------------------------------------------------------------------ */
/* One backward step u^{n+1} -> u^n (Scheme 1, Steps 1-3; Eq. (e36))          */
/* ------------------------------------------------------------------------ */

/* Exit decisions of landing points, one bit per (step, active row, q), used
 * to freeze the exit classification for finite-difference checks. */
static long exit_bit_index(const fko_problem *P, long Ja, int n, long row, int q)
{
    long Q = 1;
    for (int a = 0; a < P->d; a++) Q *= P->gh_n;
    return ((long)n * Ja + row) * Q + q;
}

static void step_impl(const fko_problem *P, int n, const long *active, long Ja,
                      const double *u_next, const double *g_next, double *u_out,
                      unsigned char *exit_rec, const unsigned char *exit_use,
                      int *cells, unsigned char *exitf)
{
    long J = fko_num_nodes(P);
    int Q = 1;
    for (int a = 0; a < P->d; a++) Q *= P->gh_n;
    for (long j = 0; j < J; j++) {
        int cls = fko_node_class(P, j);
        if (cls == 1) {
            /* exit nodes keep their exit value (1, or 0 on an FKO_FACE_EXIT0 face) */
            int i[3];
            double x[3];
            node_index(P, j, i);
            for (int a = 0; a < P->d; a++) x[a] = P->x[a][i[a]];
            u_out[j] = (double)fko_exit_value(P, x);
        }
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (long r = 0; r < Ja; r++) {
        long j = active[r];
        double sum = 0.0;
        for (int q = 0; q < Q; q++) {
            int qi[3];
            double z[3];
            split_q(P, q, qi);
            double w = tensor_weight(P, qi);
            fko_landing(P, n, j, q, z);
            int ex;
            int ev = fko_exit_value(P, z);
            if (exit_use) {
                long bi = exit_bit_index(P, Ja, n, r, q);
                ex = (exit_use[bi >> 3] >> (bi & 7)) & 1;
            } else {
                ex = ev >= 0;
            }
            if (exit_rec && ex) {
                long bi = exit_bit_index(P, Ja, n, r, q);
#pragma omp atomic
                exit_rec[bi >> 3] |= (unsigned char)(1u << (bi & 7));
            }
            if (cells) {
                for (int a = 0; a < P->d; a++)
                    cells[(r * Q + q) * P->d + a] =
                        ex ? -1 : fko_cell(P->x[a], P->n[a], z[a]);
                exitf[r * Q + q] = (unsigned char)ex;
            }
            double v = ex ? (ev == 0 ? 0.0 : 1.0) : interp(P, u_next, g_next, z, NULL);
            sum += w * v;
        }
        u_out[j] = sum;
    }
    for (long j = 0; j < J; j++)
        if (fko_node_class(P, j) == 2) u_out[j] = u_out[representative(P, j)];
}

/* One step from an arbitrary state u_next (exit nodes of the result are 1). */
int fko_step(const fko_problem *P, int n, const double *u_next, double *u_out)
{
    long J = fko_num_nodes(P);
    long Ja = fko_active_nodes(P, NULL);
    long *active = (long *)malloc(sizeof(long) * (Ja > 0 ? Ja : 1));
    double *g = (double *)malloc(sizeof(double) * J * fko_num_fields(P));
    if (!active || !g) { free(active); free(g); return -1; }
    fko_active_nodes(P, active);
    fko_slopes(P, u_next, g);
    step_impl(P, n, active, Ja, u_next, g, u_out, NULL, NULL, NULL, NULL);
    free(active);
    free(g);
    return 0;
}

/* Landing cells and exit flags of step n (layouts [Ja][Q][d] and [Ja][Q]);
 * cells of exiting landing points are -1.  The state used is u_next. */
int fko_step_cells(const fko_problem *P, int n, const double *u_next, int *cells,
                   unsigned char *exitf)
{
    long J = fko_num_nodes(P);
    long Ja = fko_active_nodes(P, NULL);
    long *active = (long *)malloc(sizeof(long) * (Ja > 0 ? Ja : 1));
    double *g = (double *)malloc(sizeof(double) * J * fko_num_fields(P));
    double *tmp = (double *)malloc(sizeof(double) * J);
    if (!active || !g || !tmp) { free(active); free(g); free(tmp); return -1; }
    fko_active_nodes(P, active);
    fko_slopes(P, u_next, g);
    step_impl(P, n, active, Ja, u_next, g, tmp, NULL, NULL, cells, exitf);
    free(active); free(g); free(tmp);
    return 0;
}

/* Terminal state chi (Section 3.2): 1 on exit nodes, 0 elsewhere. */
void fko_chi(const fko_problem *P, double *u)
{
    long J = fko_num_nodes(P);
    for (long j = 0; j < J; j++) {
        long rj = representative(P, j);
        if (fko_node_class(P, rj) != 1) {
            u[j] = 0.0;
        } else {
            int i[3];
            double x[3];
            node_index(P, rj, i);
            for (int a = 0; a < P->d; a++) x[a] = P->x[a][i[a]];
            u[j] = (double)fko_exit_value(P, x);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Whole backward pass (Eq. (e37) for one horizon)                           */
/* ------------------------------------------------------------------------ */

/* out[s * J + j] = u^{snap[s]}_j.  exit_rec / exit_use: optional bit arrays
 * of size N * Ja * Q bits (see exit_bit_index). */
int fko_solve(const fko_problem *P, const int *snap, int n_snap, double *out,
              unsigned char *exit_rec, const unsigned char *exit_use)
{
    long J = fko_num_nodes(P);
    long Ja = fko_active_nodes(P, NULL);
    long *active = (long *)malloc(sizeof(long) * (Ja > 0 ? Ja : 1));
    double *u = (double *)malloc(sizeof(double) * J);
    double *v = (double *)malloc(sizeof(double) * J);
    double *g = (double *)malloc(sizeof(double) * J * fko_num_fields(P));
    if (!active || !u || !v || !g) { free(active); free(u); free(v); free(g); return -1; }
    fko_active_nodes(P, active);
    fko_chi(P, u);
    for (int s = 0; s < n_snap; s++)
        if (snap[s] == P->n_steps) memcpy(out + (long)s * J, u, sizeof(double) * J);
    for (int n = P->n_steps - 1; n >= 0; n--) {
        fko_slopes(P, u, g);
        step_impl(P, n, active, Ja, u, g, v, exit_rec, exit_use, NULL, NULL);
        double *t = u; u = v; v = t;
        for (int s = 0; s < n_snap; s++)
            if (snap[s] == n) memcpy(out + (long)s * J, u, sizeof(double) * J);
    }
    free(active); free(u); free(v); free(g);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1 (Section 3.2): several horizons in one backward sweep          */
/* ------------------------------------------------------------------------ */

/* Horizons m[h] >= 1 (in steps, any order, repeats allowed) from the start
 * time t0: out[h * J + j] = p^{m[h]}_j of Eq. (e37), the approximate
 * probability of exiting by t0 + m[h] dt when starting from x_j at t0.
 * Algorithm 1: every column of P starts as chi; the sweep runs n = M, .., 1
 * (M = the largest horizon), and at sweep index n every column whose horizon
 * is at least n is replaced by Q Psi^{n-1} F^{n-1} of itself, i.e. takes one
 * step of Scheme 1 with the coefficients at t0 + (n-1) dt (plus the exit
 * mass).  Psi^{n-1} is the same for every column; here each column's step
 * recomputes its landing points, which gives the same values.  P->n_steps is
 * not used. */
int fko_solve_horizons(const fko_problem *P, const int *m, int n_h, double *out)
{
    long J = fko_num_nodes(P);
    long Ja = fko_active_nodes(P, NULL);
    int M = 0;
    for (int h = 0; h < n_h; h++) {
        if (m[h] < 1) return -2;
        if (m[h] > M) M = m[h];
    }
    long *active = (long *)malloc(sizeof(long) * (Ja > 0 ? Ja : 1));
    double *g = (double *)malloc(sizeof(double) * J * fko_num_fields(P));
    double *v = (double *)malloc(sizeof(double) * J);
    if (!active || !g || !v) { free(active); free(g); free(v); return -1; }
    fko_active_nodes(P, active);
    for (int h = 0; h < n_h; h++) fko_chi(P, out + (long)h * J);   /* repmat(chi, 1, M) */
    for (int n = M; n >= 1; n--) {
        for (int h = 0; h < n_h; h++) {
            if (m[h] < n) continue;                  /* columns n .. M only */
            double *col = out + (long)h * J;
            fko_slopes(P, col, g);                   /* F^{n-1} of this column */
            step_impl(P, n - 1, active, Ja, col, g, v, NULL, NULL, NULL, NULL);
            memcpy(col, v, sizeof(double) * J);
        }
    }
    free(active); free(g); free(v);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Explicit row of the step operator A_n = Q Psi^n (Eq. (e34)-(e36))          */
/* ------------------------------------------------------------------------ */

/* row[f * J + c]: coefficient of field f at node c, where field 0 is u and
 * field 1 + a is the slope along axis a; exit_mass = sum of w_q over exiting
 * landing points, so that u^n_j = exit_mass + row . [u; g]. */
int fko_assemble_row(const fko_problem *P, int n, long j, double *row, double *exit_mass)
{
    if (P->hermite == 2) return -3;   /* rows of the values and first derivatives only */
    long J = fko_num_nodes(P);
    int Q = 1;
    for (int a = 0; a < P->d; a++) Q *= P->gh_n;
    memset(row, 0, sizeof(double) * J * (P->d + 1));
    *exit_mass = 0.0;
    for (int q = 0; q < Q; q++) {
        int qi[3], k[3], corner[3], bit[3];
        double z[3], s[3], h[3];
        split_q(P, q, qi);
        double w = tensor_weight(P, qi);
        fko_landing(P, n, j, q, z);
        int ev = fko_exit_value(P, z);
        if (ev >= 0) {
            if (ev == 1) *exit_mass += w;   /* value-0 exits carry nothing */
            continue;
        }
        locate(P, z, k, s, h);
        for (int c = 0; c < (1 << P->d); c++) {
            for (int a = 0; a < P->d; a++) {
                bit[a] = (c >> (P->d - 1 - a)) & 1;
                corner[a] = k[a] + bit[a];
            }
            long node = node_linear(P, corner);
            double wv = 1.0;
            for (int a = 0; a < P->d; a++) wv = wv * H0(bit[a], s[a]);
            row[node] += w * wv;
            for (int a = 0; a < P->d; a++) {
                double ws = h[a] * H1(bit[a], s[a]);
                for (int i = 0; i < P->d; i++)
                    if (i != a) ws = ws * H0(bit[i], s[i]);
                row[(1 + a) * J + node] += w * ws;
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Adjoint of the whole pass (exit classification held fixed)               */
/* ------------------------------------------------------------------------ */

/* The slope map of Eq. (e300) is not differentiable where a divided
 * difference vanishes; its linearisation takes derivative 0 there.  A
 * difference below flat_rel (default 2^-30) of the magnitude of the two
 * values it is taken from is rounding noise of a flat stretch (equal values
 * computed along different rounding paths) and counts as vanishing, so that
 * the adjoint does not depend on the last bits of u.  flat_rel = 0 keeps only
 * exact equality.  The tests set it to show that the parameter gradient does
 * not depend on it. */
static double flat_rel = 0x1p-30;

void fko_set_flat_rel(double r) { flat_rel = r; }

double fko_get_flat_rel(void) { return flat_rel; }

static int flat_pair(double a, double b)
{
    return fabs(a - b) <= flat_rel * (fabs(a) + fabs(b));
}

/* Transpose of the PCHIP slope map along every axis, linearised at u:
 * lam[c] += sum_a sum_j mu[a][j] d g_a[j] / d u[c]. */
static void slopes_transpose(const fko_problem *P, const double *u, const double *mu,
                             double *lam)
{
    long J = fko_num_nodes(P);
    for (int ax = 0; ax < P->d; ax++) {
        for (long j = 0; j < J; j++) {
            double m = mu[ax * J + j];
            if (m == 0.0) continue;
            int i[3], il, ic, ir, kind;
            double hl, hr;
            node_index(P, j, i);
            slope_stencil(P, ax, i[ax], &il, &ic, &ir, &hl, &hr, &kind);
            int t[3];
            memcpy(t, i, sizeof(t));
            t[ax] = il; long nl = node_linear(P, t);
            t[ax] = ic; long nc = node_linear(P, t);
            t[ax] = ir; long nr = node_linear(P, t);
            if (flat_pair(u[nc], u[nl]) || flat_pair(u[nr], u[nc])) continue;
            double dl = (u[nc] - u[nl]) / hl;
            double dr = (u[nr] - u[nc]) / hr;
            if (!(dl * dr > 0.0)) continue;
            double den = (dl + dr) * (dl + dr);
            double gdl = 2.0 * dr * dr / den;   /* d g / d dl */
            double gdr = 2.0 * dl * dl / den;   /* d g / d dr */
            lam[nl] += m * (-gdl / hl);
            lam[nc] += m * (gdl / hl - gdr / hr);
            lam[nr] += m * (gdr / hr);
        }
    }
}

/* Reverse sweep of the adjoint from the stored states U[n * J + j] = u^n_j,
 * n = 0..N (the forward pass of the same problem, or any states the caller
 * supplies).  Given lam0 = dJ/du^0 (length J), returns grad = dJ/dtheta
 * (fko_num_theta entries, theta = (drift parameters, D)) and, if lamN is
 * given, dJ/du^N on active nodes. */
int fko_adjoint_states(const fko_problem *P, const double *U, const double *lam0,
                       double *grad, double *lamN, const unsigned char *exit_use)
{
    if (P->coef_kind == FKO_COEF_RUNAWAY3D) return -3;   /* state-dependent sigma: not linearised */
    for (int a = 0; a < P->d; a++)
        if (P->face[a][0] != FKO_FACE_EXIT1 || P->face[a][1] != FKO_FACE_EXIT1) return -3;
    if (P->hermite == 2) return -3;   /* the adjoint linearises the R1 interpolant */
    long J = fko_num_nodes(P);
    int N = P->n_steps;
    int nt = fko_num_theta(P);
    int Q = 1;
    for (int a = 0; a < P->d; a++) Q *= P->gh_n;
    long Ja = fko_active_nodes(P, NULL);
    long *active = (long *)malloc(sizeof(long) * (Ja > 0 ? Ja : 1));
    double *g = (double *)malloc(sizeof(double) * J * fko_num_fields(P));
    double *lam = (double *)malloc(sizeof(double) * J);
    double *mu = (double *)malloc(sizeof(double) * J * (P->d + 1));
    char *cls = (char *)malloc((size_t)J);
    if (!active || !g || !lam || !mu || !cls) {
        free(active); free(g); free(lam); free(mu); free(cls);
        return -1;
    }
    fko_active_nodes(P, active);
    for (long j = 0; j < J; j++) cls[j] = (char)fko_node_class(P, j);

    /* lam^0: only active nodes carry sensitivity; an image node's cotangent
     * belongs to the node it copies. */
    for (long j = 0; j < J; j++) lam[j] = 0.0;
    for (long j = 0; j < J; j++) {
        if (cls[j] == 0) lam[j] += lam0[j];
        else if (cls[j] == 2) {
            long rj = representative(P, j);
            if (cls[rj] == 0) lam[rj] += lam0[j];
        }
    }
    for (int k = 0; k < nt; k++) grad[k] = 0.0;

    double sq = sqrt(2.0 * P->dt);
    double S = sqrt(2.0 * P->D) * sq;
    (void)S;
    for (int n = 0; n < N; n++) {
        const double *v = U + (long)(n + 1) * J;
        fko_slopes(P, v, g);
        memset(mu, 0, sizeof(double) * J * (P->d + 1));
        double t = P->t0 + (double)n * P->dt;
        double gacc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : gacc[:8])
        for (long r = 0; r < Ja; r++) {
            long j = active[r];
            double L = lam[j];
            if (L == 0.0) continue;
            int ij[3];
            double xj[3];
            node_index(P, j, ij);
            for (int a = 0; a < P->d; a++) xj[a] = P->x[a][ij[a]];
            for (int q = 0; q < Q; q++) {
                int qi[3], k[3], corner[3], bit[3];
                double z[3], s[3], h[3], an[3], dz[8 * 3], grd[3];
                split_q(P, q, qi);
                double w = tensor_weight(P, qi);
                fko_landing(P, n, j, q, z);
                int ex;
                if (exit_use) {
                    long bi = exit_bit_index(P, Ja, n, r, q);
                    ex = (exit_use[bi >> 3] >> (bi & 7)) & 1;
                } else {
                    ex = fko_is_exit_point(P, z);
                }
                if (ex) continue;
                double Lw = L * w;
                /* scatter: transpose of the interpolation row */
                locate(P, z, k, s, h);
                for (int c = 0; c < (1 << P->d); c++) {
                    for (int a = 0; a < P->d; a++) {
                        bit[a] = (c >> (P->d - 1 - a)) & 1;
                        corner[a] = k[a] + bit[a];
                    }
                    long node = node_linear(P, corner);
                    double wv = 1.0;
                    for (int a = 0; a < P->d; a++) wv = wv * H0(bit[a], s[a]);
#pragma omp atomic
                    mu[node] += Lw * wv;
                    for (int a = 0; a < P->d; a++) {
                        double ws = h[a] * H1(bit[a], s[a]);
                        for (int i = 0; i < P->d; i++)
                            if (i != a) ws = ws * H0(bit[i], s[i]);
#pragma omp atomic
                        mu[(1 + a) * J + node] += Lw * ws;
                    }
                }
                /* parameter sensitivity through the landing point */
                interp(P, v, g, z, grd);
                for (int a = 0; a < P->d; a++) an[a] = P->gh_a[qi[a]];
                dz_dtheta(P, t, xj, an, dz);
                for (int kk = 0; kk < nt; kk++) {
                    double sdot = 0.0;
                    for (int a = 0; a < P->d; a++) sdot += grd[a] * dz[kk * 3 + a];
                    gacc[kk] += Lw * sdot;
                }
            }
        }
        for (int kk = 0; kk < nt; kk++) grad[kk] += gacc[kk];
        /* lam^{n+1} = mu_u + sum_a J_{F_a}(v)^T mu_a */
        for (long j = 0; j < J; j++) lam[j] = mu[j];
        slopes_transpose(P, v, mu + J, lam);
        /* exit nodes hold the constant 1; image nodes pass to their originals */
        for (long j = 0; j < J; j++) {
            if (cls[j] == 2) {
                long rj = representative(P, j);
                if (cls[rj] == 0) lam[rj] += lam[j];
                lam[j] = 0.0;
            }
        }
        for (long j = 0; j < J; j++)
            if (cls[j] != 0) lam[j] = 0.0;
    }
    if (lamN) memcpy(lamN, lam, sizeof(double) * J);
    free(active); free(g); free(lam); free(mu); free(cls);
    return 0;
}

/* Every state of the backward pass: U[n * J + j] = u^n_j, n = 0..N. */
int fko_solve_all(const fko_problem *P, double *U, const unsigned char *exit_use)
{
    long J = fko_num_nodes(P);
    int N = P->n_steps;
    long Ja = fko_active_nodes(P, NULL);
    long *active = (long *)malloc(sizeof(long) * (Ja > 0 ? Ja : 1));
    double *g = (double *)malloc(sizeof(double) * J * fko_num_fields(P));
    if (!active || !g) { free(active); free(g); return -1; }
    fko_active_nodes(P, active);
    fko_chi(P, U + (long)N * J);
    for (int n = N - 1; n >= 0; n--) {
        fko_slopes(P, U + (long)(n + 1) * J, g);
        step_impl(P, n, active, Ja, U + (long)(n + 1) * J, g, U + (long)n * J,
                  NULL, exit_use, NULL, NULL);
    }
    free(active); free(g);
    return 0;
}

/* Adjoint of the whole pass: the forward pass keeping every u^n (memory
 * (N + 1) J doubles), then the reverse sweep. */
int fko_adjoint(const fko_problem *P, const double *lam0, double *grad, double *lamN,
                const unsigned char *exit_use)
{
    long J = fko_num_nodes(P);
    double *U = (double *)malloc(sizeof(double) * J * (long)(P->n_steps + 1));
    if (!U) return -1;
    int rc = fko_solve_all(P, U, exit_use);
    if (rc == 0) rc = fko_adjoint_states(P, U, lam0, grad, lamN, exit_use);
    free(U);
    return rc;
}
