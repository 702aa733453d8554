/*
 * bem_oracle.c -- plain, slow, FP64 reference of the Laplace-domain collocation BEM
 * entries and dense products.  TEST INFRASTRUCTURE ONLY: tests, the smoke check and the
 * CPU baseline of the benchmark call it; the product library never links or calls it.
 *
 * What it computes (Keshava & Schanz, "A 3D-ACA accelerated time domain BEM for
 * elastodynamics"):
 *   - U(r, s): Laplace transform of the full-space displacement tensor of Appendix A,
 *     eq. (A.2), taken with an impulse source:
 *         4 pi rho U_ij = f0_ij I1 + f1_ij e1 + f2_ij e2,
 *         f0 = (3 rh_i rh_j - d_ij)/r, f1 = rh_i rh_j/(r c1^2), f2 = (d_ij - rh_i rh_j)/(r c2^2),
 *         e_a = exp(-s r / c_a),  I1 = int_{1/c1}^{1/c2} lam exp(-s lam r) dlam.
 *     (In the printed f0, f1, f2 the symbol r_i is the unit vector; dimensions require it.)
 *   - T(x, y, n, s): traction at y (normal n) of the field U_i.(y - x) of a unit load in
 *     direction i at x, from the stress law of Sec. 2.1,
 *         sigma = rho (c1^2 - 2 c2^2) div(u) I + rho c2^2 (grad u + grad u^T),  t = sigma n.
 *     The double layer acts as (K u)_i = sum_j int T_ij u_j (eq. (DLP)).
 *   - Collocation entries at element centroids with piecewise-constant trial functions
 *     (eq. (discrVK), collocation points at midpoints, Sec. 2.3):
 *         V[i,j](s) = int_{gamma_j} U(y - x_i, s) dy,   K[i,j](s) = PV int_{gamma_j} T dy.
 *   - Quadrature (Sec. 2.3 names Duffy for the singular collocation integrals; the rest
 *     is this project's reading, identical on both sides of every parity test):
 *       regular pair : 7-point degree-5 triangle rule;
 *       near pair    : the same rule on 4^m congruent sub-triangles, m = 2 if
 *                      |x_i - c_j| < r1 * lmax_j, m = 1 if < r2 * lmax_j (switchable);
 *       self pair V  : polar Duffy about the centroid, 3 sub-triangles, n_theta x n_rho
 *                      Gauss-Legendre points;
 *       self pair K  : Cauchy principal value in the same polar coordinates with the
 *                      leading 1/rho^2 part g(theta) = c2^2/(4 pi c1^2) (rh_i n_j - rh_j n_i)
 *                      integrated analytically in rho (its log terms cancel over 2 pi).
 *   - op 2 adds the free term C = I/2 of eq. (SBIE) at smooth points to K.
 *   - ops 4, 5, 6: the double layer against the continuous piecewise-linear shape functions
 *     of the Dirichlet data (eqs. (subspace), (basis), K of eq. (discrVK) with phi_l): the
 *     integrand T of element j weighted by the barycentric coordinate lambda_v(y) of its
 *     vertex v = op - 4, with the same rules; in the self pair the principal value is taken
 *     with the leading part weighted by lambda_v at the centroid (1/3), the remainder
 *     T (lambda_v(y) - 1/3) being weakly singular.  The linear-basis operator sums these over
 *     the elements sharing a node.
 *   - oracle_adjoint_v / oracle_adjoint_k: the gradient of Re sum_l w_l^T A(s_l) x_l (A = V,
 *     K or I/2 + K) with respect to the node coordinates and the material, the pair classes
 *     held fixed: regular and near pairs by the chain rule through the quadrature points, the
 *     normal, the area and the collocation point; self pairs as the derivative of the
 *     (principal-value) integral, or by central differences of the polar rule.
 *
 * Everything is written per entry, per quadrature point, per frequency; no blocking,
 * no reuse across frequencies, no shared tables with the GPU library.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

typedef struct {
    double rho, c1, c2;
} material;

typedef struct {
    int near_on;
    double r1, r2;
    int self_nt, self_nr;
} quadopts;

/* ---------------------------------------------------------------- quadrature rules */

/* 7-point degree-5 rule on a triangle in barycentric coordinates; weights sum to 1. */
void oracle_tri7(double *bary, double *w)
{
    const double s15 = sqrt(15.0);
    const double a = (6.0 - s15) / 21.0, b = (6.0 + s15) / 21.0;
    const double wa = (155.0 - s15) / 1200.0, wb = (155.0 + s15) / 1200.0;
    double B[7][3] = {
        {1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0},
        {a, a, 1.0 - 2.0 * a}, {a, 1.0 - 2.0 * a, a}, {1.0 - 2.0 * a, a, a},
        {b, b, 1.0 - 2.0 * b}, {b, 1.0 - 2.0 * b, b}, {1.0 - 2.0 * b, b, b},
    };
    double W[7] = {9.0 / 40.0, wa, wa, wa, wb, wb, wb};
    for (int q = 0; q < 7; ++q) {
        for (int k = 0; k < 3; ++k) bary[3 * q + k] = B[q][k];
        w[q] = W[q];
    }
}

/* Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on the three-term
 * Legendre recurrence. */
void oracle_gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        /* recompute derivative at the converged node */
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        if (n == 1) { p1 = z; p0 = 1.0; }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* ------------------------------------------------------------------ the kernel */

/* int_{1/c1}^{1/c2} lam^p exp(-alpha lam) dlam for p = 1, 2 and alpha = s r. */
static cplx lam_integral(int p, cplx alpha, double c1, double c2)
{
    const double a = 1.0 / c1, b = 1.0 / c2;
    if (cabs(alpha) * b < 2.0) {
        /* Taylor series of the exponential, integrated term by term */
        cplx sum = 0.0, term = 1.0; /* term = (-alpha)^n / n! */
        for (int n = 0; n < 400; ++n) {
            double e = n + p + 1.0;
            cplx add = term * (pow(b, e) - pow(a, e)) / e;
            sum += add;
            if (n > 4 && cabs(add) < 1e-19 * cabs(sum)) break;
            term *= -alpha / (n + 1.0);
        }
        return sum;
    }
    /* closed form of the antiderivative F(lam) = -exp(-alpha lam) * poly */
    cplx Fa, Fb;
    if (p == 1) {
        Fb = -cexp(-alpha * b) * (b / alpha + 1.0 / (alpha * alpha));
        Fa = -cexp(-alpha * a) * (a / alpha + 1.0 / (alpha * alpha));
    } else {
        Fb = -cexp(-alpha * b) * (b * b / alpha + 2.0 * b / (alpha * alpha) + 2.0 / (alpha * alpha * alpha));
        Fa = -cexp(-alpha * a) * (a * a / alpha + 2.0 * a / (alpha * alpha) + 2.0 / (alpha * alpha * alpha));
    }
    return Fb - Fa;
}

/* U(y - x, s), 3x3 row-major. */
static void kernel_U(const double *rv, cplx s, const material *m, cplx *U)
{
    double r = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
    double rh[3] = {rv[0] / r, rv[1] / r, rv[2] / r};
    cplx I1 = lam_integral(1, s * r, m->c1, m->c2);
    cplx e1 = cexp(-s * r / m->c1), e2 = cexp(-s * r / m->c2);
    double pref = 1.0 / (4.0 * M_PI * m->rho);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double dij = (i == j) ? 1.0 : 0.0;
            double P = rh[i] * rh[j];
            double f0 = (3.0 * P - dij) / r;
            double f1 = P / (r * m->c1 * m->c1);
            double f2 = (dij - P) / (r * m->c2 * m->c2);
            U[3 * i + j] = pref * (f0 * I1 + f1 * e1 + f2 * e2);
        }
}

/* Gradient dU_ij/dy_k (r = y - x) by the product rule on the form of kernel_U. */
static void kernel_gradU(const double *rv, cplx s, const material *m, cplx *G /* [i][j][k] */)
{
    double r = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
    double rh[3] = {rv[0] / r, rv[1] / r, rv[2] / r};
    double c1 = m->c1, c2 = m->c2;
    cplx I1 = lam_integral(1, s * r, c1, c2);
    cplx I2 = lam_integral(2, s * r, c1, c2);
    cplx e1 = cexp(-s * r / c1), e2 = cexp(-s * r / c2);
    /* radial scalar factors and their r-derivatives */
    cplx a = I1 / r;
    cplx da = (-s * I2) / r - I1 / (r * r);               /* dI1/dr = -s I2 */
    cplx b = e1 / (c1 * c1 * r);
    cplx db = e1 / (c1 * c1) * (-(s / c1) / r - 1.0 / (r * r));
    cplx c = e2 / (c2 * c2 * r);
    cplx dc = e2 / (c2 * c2) * (-(s / c2) / r - 1.0 / (r * r));
    double pref = 1.0 / (4.0 * M_PI * m->rho);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) {
                double dij = (i == j) ? 1.0 : 0.0, dik = (i == k) ? 1.0 : 0.0, djk = (j == k) ? 1.0 : 0.0;
                double P = rh[i] * rh[j];
                double dP = (dik * rh[j] + djk * rh[i] - 2.0 * rh[i] * rh[j] * rh[k]) / r;
                cplx v = (3.0 * P - dij) * da * rh[k] + 3.0 * a * dP
                       + P * db * rh[k] + b * dP
                       + (dij - P) * dc * rh[k] - c * dP;
                G[9 * i + 3 * j + k] = pref * v;
            }
}

/* T_ij(x, y, n, s): traction component j at y of the field of a unit load in direction i. */
static void kernel_T(const double *x, const double *y, const double *n, cplx s, const material *m, cplx *T)
{
    double rv[3] = {y[0] - x[0], y[1] - x[1], y[2] - x[2]};
    cplx G[27];
    kernel_gradU(rv, s, m, G);
    double lam = m->rho * (m->c1 * m->c1 - 2.0 * m->c2 * m->c2);
    double mu = m->rho * m->c2 * m->c2;
    for (int i = 0; i < 3; ++i) {
        /* displacement field u_j = U_ij, gradient du_j/dy_k = G[i][j][k] */
        cplx div = G[9 * i + 0] + G[9 * i + 4] + G[9 * i + 8];
        for (int j = 0; j < 3; ++j) {
            cplx t = 0.0;
            for (int k = 0; k < 3; ++k) {
                cplx eps = 0.5 * (G[9 * i + 3 * j + k] + G[9 * i + 3 * k + j]);
                cplx sig = ((j == k) ? lam * div : 0.0) + 2.0 * mu * eps;
                t += sig * n[k];
            }
            T[3 * i + j] = t;
        }
    }
}

int oracle_kernel_point(int which, const double *x, const double *y, const double *n,
                        double sr, double si, double rho, double cp, double cs, double *out)
{
    material m = {rho, cp, cs};
    cplx s = sr + I * si;
    cplx R[9];
    if (which == 0) {
        double rv[3] = {y[0] - x[0], y[1] - x[1], y[2] - x[2]};
        kernel_U(rv, s, &m, R);
    } else if (which == 1) {
        kernel_T(x, y, n, s, &m, R);
    } else {
        return -1;
    }
    for (int k = 0; k < 9; ++k) {
        out[2 * k] = creal(R[k]);
        out[2 * k + 1] = cimag(R[k]);
    }
    return 0;
}

/* --------------------------------------------------------------- element geometry */

typedef struct {
    double v[3][3];   /* vertices */
    double c[3];      /* centroid */
    double n[3];      /* unit normal (v1-v0)x(v2-v0) */
    double area;
    double lmax2;     /* squared longest edge */
} element;

static void make_element(const double *nodes, const int32_t *tri, element *e)
{
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 3; ++k) e->v[a][k] = nodes[3 * (int64_t)tri[a] + k];
    for (int k = 0; k < 3; ++k) e->c[k] = (e->v[0][k] + e->v[1][k] + e->v[2][k]) / 3.0;
    double u[3], w[3], nn[3];
    for (int k = 0; k < 3; ++k) { u[k] = e->v[1][k] - e->v[0][k]; w[k] = e->v[2][k] - e->v[0][k]; }
    nn[0] = u[1] * w[2] - u[2] * w[1];
    nn[1] = u[2] * w[0] - u[0] * w[2];
    nn[2] = u[0] * w[1] - u[1] * w[0];
    double len = sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
    e->area = 0.5 * len;
    for (int k = 0; k < 3; ++k) e->n[k] = nn[k] / len;
    double l2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        int b = (a + 1) % 3;
        double dx = e->v[b][0] - e->v[a][0], dy = e->v[b][1] - e->v[a][1], dz = e->v[b][2] - e->v[a][2];
        double q = dx * dx + dy * dy + dz * dz;
        if (q > l2) l2 = q;
    }
    e->lmax2 = l2;
}

/* ----------------------------------------------------------------- integration */

typedef struct {
    const element *el;     /* all elements */
    material mat;
    quadopts qo;
    double tri_bary[21], tri_w[7];
    double gl_t[64], gl_tw[64], gl_r[64], gl_rw[64];
} ctx;

/* Barycentric coordinate of vertex v of element e at a point y of its plane:
 * lambda_v(y) = n . ((P_{v+1} - y) x (P_{v+2} - y)) / (2 A).  vw < 0: weight 1. */
static double bary_weight(const element *e, int vw, const double *y)
{
    if (vw < 0) return 1.0;
    const double *p1 = e->v[(vw + 1) % 3], *p2 = e->v[(vw + 2) % 3];
    double a[3], b[3];
    for (int k = 0; k < 3; ++k) { a[k] = p1[k] - y[k]; b[k] = p2[k] - y[k]; }
    double cr[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    return (e->n[0] * cr[0] + e->n[1] * cr[1] + e->n[2] * cr[2]) / (2.0 * e->area);
}

/* integrand value at y for collocation point x and element normal n (op 0: U, else T) */
static void integrand(int op, const double *x, const double *y, const double *n, cplx s, const material *m, cplx *R)
{
    if (op == 0) {
        double rv[3] = {y[0] - x[0], y[1] - x[1], y[2] - x[2]};
        kernel_U(rv, s, m, R);
    } else {
        kernel_T(x, y, n, s, m, R);
    }
}

/* 7-point rule over the triangle (p0, p1, p2) of area A, accumulated into acc. */
static void tri_rule(const ctx *C, int op, const double *x, const double *p0, const double *p1, const double *p2,
                     double A, const double *n, cplx s, const element *par, int vw, cplx *acc)
{
    for (int q = 0; q < 7; ++q) {
        const double *B = &C->tri_bary[3 * q];
        double y[3];
        for (int k = 0; k < 3; ++k) y[k] = B[0] * p0[k] + B[1] * p1[k] + B[2] * p2[k];
        cplx R[9];
        integrand(op, x, y, n, s, &C->mat, R);
        const double lw = bary_weight(par, vw, y);
        for (int t = 0; t < 9; ++t) acc[t] += C->tri_w[q] * A * lw * R[t];
    }
}

/* 7-point rule on the 4^m sub-triangles obtained by repeated edge-midpoint splitting. */
static void subdivided_rule(const ctx *C, int op, const double *x, const double *p0, const double *p1,
                            const double *p2, double A, const double *n, cplx s, int m, const element *par, int vw,
                            cplx *acc)
{
    if (m == 0) {
        tri_rule(C, op, x, p0, p1, p2, A, n, s, par, vw, acc);
        return;
    }
    double m01[3], m12[3], m20[3];
    for (int k = 0; k < 3; ++k) {
        m01[k] = 0.5 * (p0[k] + p1[k]);
        m12[k] = 0.5 * (p1[k] + p2[k]);
        m20[k] = 0.5 * (p2[k] + p0[k]);
    }
    subdivided_rule(C, op, x, p0, m01, m20, 0.25 * A, n, s, m - 1, par, vw, acc);
    subdivided_rule(C, op, x, m01, p1, m12, 0.25 * A, n, s, m - 1, par, vw, acc);
    subdivided_rule(C, op, x, m20, m12, p2, 0.25 * A, n, s, m - 1, par, vw, acc);
    subdivided_rule(C, op, x, m01, m12, m20, 0.25 * A, n, s, m - 1, par, vw, acc);
}

/* Self element: polar coordinates about the centroid x on the three sub-triangles
 * (x, v_a, v_b); theta is measured from the foot of the perpendicular onto edge v_a v_b. */
static void self_rule(const ctx *C, int op, const element *e, cplx s, int vw, cplx *acc)
{
    const double *x = e->c;
    const double *n = e->n;
    const material *m = &C->mat;
    const double lx = bary_weight(e, vw, x);  /* weight of the leading part (1/3, or 1) */
    const double gpref = (m->c2 * m->c2) / (4.0 * M_PI * m->c1 * m->c1);
    for (int a = 0; a < 3; ++a) {
        const double *va = e->v[a], *vb = e->v[(a + 1) % 3];
        double t[3], le = 0.0;
        for (int k = 0; k < 3; ++k) { t[k] = vb[k] - va[k]; le += t[k] * t[k]; }
        le = sqrt(le);
        for (int k = 0; k < 3; ++k) t[k] /= le;
        double proj = 0.0;
        for (int k = 0; k < 3; ++k) proj += (x[k] - va[k]) * t[k];
        double foot[3], p[3], d = 0.0;
        for (int k = 0; k < 3; ++k) { foot[k] = va[k] + proj * t[k]; p[k] = foot[k] - x[k]; d += p[k] * p[k]; }
        d = sqrt(d);
        for (int k = 0; k < 3; ++k) p[k] /= d;
        double sa = 0.0, sb = 0.0;
        for (int k = 0; k < 3; ++k) { sa += (va[k] - foot[k]) * t[k]; sb += (vb[k] - foot[k]) * t[k]; }
        double ta = atan2(sa, d), tb = atan2(sb, d);
        for (int it = 0; it < C->qo.self_nt; ++it) {
            double th = 0.5 * (ta + tb) + 0.5 * (tb - ta) * C->gl_t[it];
            double wth = 0.5 * (tb - ta) * C->gl_tw[it];
            double R = d / cos(th);
            double dir[3];
            for (int k = 0; k < 3; ++k) dir[k] = cos(th) * p[k] + sin(th) * t[k];
            cplx g[9];
            if (op != 0) {
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) g[3 * i + j] = gpref * (dir[i] * n[j] - dir[j] * n[i]);
                for (int q = 0; q < 9; ++q) acc[q] += wth * lx * g[q] * log(R);
            }
            for (int ir = 0; ir < C->qo.self_nr; ++ir) {
                double rho = 0.5 * R * (1.0 + C->gl_r[ir]);
                double wr = 0.5 * R * C->gl_rw[ir];
                double y[3];
                for (int k = 0; k < 3; ++k) y[k] = x[k] + rho * dir[k];
                cplx Rv[9];
                integrand(op, x, y, n, s, m, Rv);
                const double ly = bary_weight(e, vw, y);
                for (int q = 0; q < 9; ++q) {
                    cplx f = rho * ly * Rv[q];
                    if (op != 0) f -= lx * g[q] / rho;
                    acc[q] += wth * wr * f;
                }
            }
        }
    }
}

/* One 3x3 entry: collocation at the centroid of element i, element j, frequency s. */
static void entry(const ctx *C, int op, int64_t i, int64_t j, cplx s, cplx *out)
{
    for (int t = 0; t < 9; ++t) out[t] = 0.0;
    const element *ei = &C->el[i], *ej = &C->el[j];
    int kop = (op == 0) ? 0 : 1;
    int vw = (op >= 4 && op <= 6) ? op - 4 : -1;  /* linear shape function of vertex vw */
    if (i == j) {
        self_rule(C, kop, ej, s, vw, out);
    } else {
        int m = 0;
        if (C->qo.near_on) {
            double dx = ei->c[0] - ej->c[0], dy = ei->c[1] - ej->c[1], dz = ei->c[2] - ej->c[2];
            double d2 = dx * dx + dy * dy + dz * dz;
            if (d2 < C->qo.r1 * C->qo.r1 * ej->lmax2) m = 2;
            else if (d2 < C->qo.r2 * C->qo.r2 * ej->lmax2) m = 1;
        }
        subdivided_rule(C, kop, ei->c, ej->v[0], ej->v[1], ej->v[2], ej->area, ej->n, s, m, ej, vw, out);
    }
    if (op == 2 && i == j) {
        out[0] += 0.5;
        out[4] += 0.5;
        out[8] += 0.5;
    }
}

static int setup(ctx *C, const double *nodes, int64_t n_nodes, const int32_t *tris, int64_t K,
                 double rho, double cp, double cs, int near_on, double r1, double r2, int self_nt, int self_nr)
{
    if (K < 1 || self_nt < 1 || self_nt > 64 || self_nr < 1 || self_nr > 64) return -1;
    for (int64_t e = 0; e < 3 * K; ++e)
        if (tris[e] < 0 || tris[e] >= n_nodes) return -2;
    element *el = (element *)malloc(sizeof(element) * (size_t)K);
    if (!el) return -3;
    for (int64_t e = 0; e < K; ++e) make_element(nodes, tris + 3 * e, &el[e]);
    C->el = el;
    C->mat.rho = rho;
    C->mat.c1 = cp;
    C->mat.c2 = cs;
    C->qo.near_on = near_on;
    C->qo.r1 = r1;
    C->qo.r2 = r2;
    C->qo.self_nt = self_nt;
    C->qo.self_nr = self_nr;
    oracle_tri7(C->tri_bary, C->tri_w);
    oracle_gauss_legendre(self_nt, C->gl_t, C->gl_tw);
    oracle_gauss_legendre(self_nr, C->gl_r, C->gl_rw);
    return 0;
}

/* Entries out[e] = ENTRY(op, ii[e], jj[e], ll[e]) as [n][9][re, im]. */
int oracle_entries(const double *nodes, int64_t n_nodes, const int32_t *tris, int64_t K,
                   double rho, double cp, double cs, const double *s, int32_t L,
                   int op, int near_on, double r1, double r2, int self_nt, int self_nr,
                   int64_t n, const int32_t *ii, const int32_t *jj, const int32_t *ll, double *out)
{
    ctx C;
    int rc = setup(&C, nodes, n_nodes, tris, K, rho, cp, cs, near_on, r1, r2, self_nt, self_nr);
    if (rc) return rc;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
    for (int64_t e = 0; e < n; ++e) {
        if (ii[e] < 0 || ii[e] >= K || jj[e] < 0 || jj[e] >= K || ll[e] < 0 || ll[e] >= L) { bad = 1; continue; }
        cplx R[9];
        entry(&C, op, ii[e], jj[e], s[2 * ll[e]] + I * s[2 * ll[e] + 1], R);
        for (int t = 0; t < 9; ++t) {
            out[18 * e + 2 * t] = creal(R[t]);
            out[18 * e + 2 * t + 1] = cimag(R[t]);
        }
    }
    free((void *)C.el);
    return bad ? -4 : 0;
}

/* Dense product on selected rows: y[r][l][3*q + a] = sum_j sum_b ENTRY(rows[q], j, l)[a][b]
 * x[r][l][3 j + b] for every right-hand side r and frequency l.
 * x: [nrhs][L][3K] complex, y: [nrhs][L][3*nrows] complex (interleaved re, im). */
int oracle_matvec_rows(const double *nodes, int64_t n_nodes, const int32_t *tris, int64_t K,
                       double rho, double cp, double cs, const double *s, int32_t L,
                       int op, int near_on, double r1, double r2, int self_nt, int self_nr,
                       int64_t nrows, const int32_t *rows, int32_t nrhs, const double *x, double *y)
{
    ctx C;
    int rc = setup(&C, nodes, n_nodes, tris, K, rho, cp, cs, near_on, r1, r2, self_nt, self_nr);
    if (rc) return rc;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) collapse(2) reduction(| : bad)
    for (int64_t q = 0; q < nrows; ++q) {
        for (int32_t l = 0; l < L; ++l) {
            int64_t i = rows[q];
            if (i < 0 || i >= K) { bad = 1; continue; }
            cplx s_l = s[2 * l] + I * s[2 * l + 1];
            cplx acc[64][3];
            for (int r = 0; r < nrhs && r < 64; ++r) acc[r][0] = acc[r][1] = acc[r][2] = 0.0;
            for (int64_t j = 0; j < K; ++j) {
                cplx E[9];
                entry(&C, op, i, j, s_l, E);
                for (int r = 0; r < nrhs && r < 64; ++r) {
                    const double *xv = x + 2 * (((int64_t)r * L + l) * 3 * K + 3 * j);
                    cplx xb[3] = {xv[0] + I * xv[1], xv[2] + I * xv[3], xv[4] + I * xv[5]};
                    for (int a = 0; a < 3; ++a)
                        acc[r][a] += E[3 * a + 0] * xb[0] + E[3 * a + 1] * xb[1] + E[3 * a + 2] * xb[2];
                }
            }
            for (int r = 0; r < nrhs && r < 64; ++r)
                for (int a = 0; a < 3; ++a) {
                    double *yv = y + 2 * (((int64_t)r * L + l) * 3 * nrows + 3 * q + a);
                    yv[0] = creal(acc[r][a]);
                    yv[1] = cimag(acc[r][a]);
                }
        }
    }
    free((void *)C.el);
    if (nrhs > 64) return -5;
    return bad ? -4 : 0;
}

/* Layer integrals from arbitrary field points (not on the boundary):
 * out[e] = int_{gamma_jj[e]} kernel(pts[pp[e]], y) dy, kernel U (op 0) or T (op 1),
 * with the regular rule, or the subdivided rule when near_on and the point is close. */
int oracle_point_entries(const double *nodes, int64_t n_nodes, const int32_t *tris, int64_t K,
                         double rho, double cp, double cs, const double *s, int32_t L,
                         int op, int near_on, double r1, double r2,
                         int64_t npts, const double *pts,
                         int64_t n, const int32_t *pp, const int32_t *jj, const int32_t *ll, double *out)
{
    ctx C;
    int rc = setup(&C, nodes, n_nodes, tris, K, rho, cp, cs, near_on, r1, r2, 8, 8);
    if (rc) return rc;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
    for (int64_t e = 0; e < n; ++e) {
        if (pp[e] < 0 || pp[e] >= npts || jj[e] < 0 || jj[e] >= K || ll[e] < 0 || ll[e] >= L) { bad = 1; continue; }
        const double *x = pts + 3 * (int64_t)pp[e];
        const element *ej = &C.el[jj[e]];
        cplx s_l = s[2 * ll[e]] + I * s[2 * ll[e] + 1];
        int m = 0;
        if (near_on) {
            double dx = x[0] - ej->c[0], dy = x[1] - ej->c[1], dz = x[2] - ej->c[2];
            double d2 = dx * dx + dy * dy + dz * dz;
            if (d2 < r1 * r1 * ej->lmax2) m = 2;
            else if (d2 < r2 * r2 * ej->lmax2) m = 1;
        }
        cplx R[9];
        for (int t = 0; t < 9; ++t) R[t] = 0.0;
        subdivided_rule(&C, op == 0 ? 0 : 1, x, ej->v[0], ej->v[1], ej->v[2], ej->area, ej->n, s_l, m, ej, -1, R);
        for (int t = 0; t < 9; ++t) {
            out[18 * e + 2 * t] = creal(R[t]);
            out[18 * e + 2 * t + 1] = cimag(R[t]);
        }
    }
    free((void *)C.el);
    return bad ? -4 : 0;
}

/* ------------------------------------------------------------ adjoint of V */

/* dU_ab/dc1 and dU_ab/dc2 (c1 = c_p, c2 = c_s) by differentiating the form of kernel_U:
 * dI1/dc1 = e1 / c1^3 and dI1/dc2 = -e2 / c2^3 (the limits of the lambda-integral move),
 * d(1/c^2)/dc = -2/c^3, d exp(-s r / c)/dc = exp(-s r / c) s r / c^2. */
static void kernel_dU_dc(const double *rv, cplx s, const material *m, cplx *D1, cplx *D2)
{
    double r = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
    double rh[3] = {rv[0] / r, rv[1] / r, rv[2] / r};
    double c1 = m->c1, c2 = m->c2;
    cplx e1 = cexp(-s * r / c1), e2 = cexp(-s * r / c2);
    double pref = 1.0 / (4.0 * M_PI * m->rho);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double dij = (i == j) ? 1.0 : 0.0;
            double P = rh[i] * rh[j];
            double f0 = (3.0 * P - dij) / r;
            double f1 = P / (r * c1 * c1);
            double f2 = (dij - P) / (r * c2 * c2);
            D1[3 * i + j] = pref * (f0 * e1 / (c1 * c1 * c1) - 2.0 * f1 / c1 * e1 + f1 * e1 * s * r / (c1 * c1));
            D2[3 * i + j] = pref * (-f0 * e2 / (c2 * c2 * c2) - 2.0 * f2 / c2 * e2 + f2 * e2 * s * r / (c2 * c2));
        }
}

/* sum over r, l of w[r][l][3 i .. 3 i + 3]^T E x[r][l][3 j .. 3 j + 3] for one 3x3 block E(l) */
static cplx contract(const cplx *E, const double *w, const double *x, int64_t K, int32_t L, int32_t nrhs,
                     int32_t l, int64_t i, int64_t j)
{
    cplx sum = 0.0;
    for (int r = 0; r < nrhs; ++r) {
        const double *wv = w + 2 * (((int64_t)r * L + l) * 3 * K + 3 * i);
        const double *xv = x + 2 * (((int64_t)r * L + l) * 3 * K + 3 * j);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                sum += (wv[2 * a] + I * wv[2 * a + 1]) * E[3 * a + b] * (xv[2 * b] + I * xv[2 * b + 1]);
    }
    return sum;
}

/* Barycentric coordinates, with respect to the parent's vertices, of the vertices of the 4^m
 * sub-triangles of the edge-midpoint splitting, in the order subdivided_rule visits them:
 * out[t][b][a] is coordinate a of vertex b of sub-triangle t.  Returns the count 4^m. */
static int sub_triangles(const double *b0, const double *b1, const double *b2, int m, double (*out)[3][3], int n)
{
    if (m == 0) {
        for (int a = 0; a < 3; ++a) {
            out[n][0][a] = b0[a];
            out[n][1][a] = b1[a];
            out[n][2][a] = b2[a];
        }
        return n + 1;
    }
    double m01[3], m12[3], m20[3];
    for (int a = 0; a < 3; ++a) {
        m01[a] = 0.5 * (b0[a] + b1[a]);
        m12[a] = 0.5 * (b1[a] + b2[a]);
        m20[a] = 0.5 * (b2[a] + b0[a]);
    }
    n = sub_triangles(b0, m01, m20, m - 1, out, n);
    n = sub_triangles(m01, b1, m12, m - 1, out, n);
    n = sub_triangles(m20, m12, b2, m - 1, out, n);
    return sub_triangles(m01, m12, m20, m - 1, out, n);
}

/* Self pair of the single layer, differentiated as an integral: with the collocation point
 * x = (v_0 + v_1 + v_2) / 3 and y = sum_a lambda_a(y) v_a on the element,
 *   d/dv_a int U(y - x) dy = int grad U(y - x) (lambda_a(y) - 1/3) dy + (dA/dv_a / A) int U dy,
 *   d/dc int U dy = int dU/dc dy,
 * integrated with the polar rule of self_rule (the first integrand is O(1/|y - x|)).  Adds the
 * contraction with w, x at (l, element j) to val (complex), gv[a][k] (Re) and gc[2] (Re). */
static void self_grad(const ctx *C, const element *e, cplx s, const double *w, const double *x, int64_t K,
                      int32_t L, int32_t nrhs, int32_t l, int64_t j, const double dA[3][3], cplx *val,
                      double gv[3][3], double gc[2])
{
    const double *xc = e->c;
    cplx vsum = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double *va = e->v[a], *vb = e->v[(a + 1) % 3];
        double t[3], le = 0.0;
        for (int k = 0; k < 3; ++k) { t[k] = vb[k] - va[k]; le += t[k] * t[k]; }
        le = sqrt(le);
        for (int k = 0; k < 3; ++k) t[k] /= le;
        double proj = 0.0;
        for (int k = 0; k < 3; ++k) proj += (xc[k] - va[k]) * t[k];
        double foot[3], p[3], d = 0.0;
        for (int k = 0; k < 3; ++k) { foot[k] = va[k] + proj * t[k]; p[k] = foot[k] - xc[k]; d += p[k] * p[k]; }
        d = sqrt(d);
        for (int k = 0; k < 3; ++k) p[k] /= d;
        double sa = 0.0, sb = 0.0;
        for (int k = 0; k < 3; ++k) { sa += (va[k] - foot[k]) * t[k]; sb += (vb[k] - foot[k]) * t[k]; }
        double ta = atan2(sa, d), tb = atan2(sb, d);
        for (int it = 0; it < C->qo.self_nt; ++it) {
            double th = 0.5 * (ta + tb) + 0.5 * (tb - ta) * C->gl_t[it];
            double wth = 0.5 * (tb - ta) * C->gl_tw[it];
            double R = d / cos(th);
            double dir[3];
            for (int k = 0; k < 3; ++k) dir[k] = cos(th) * p[k] + sin(th) * t[k];
            for (int ir = 0; ir < C->qo.self_nr; ++ir) {
                double rho = 0.5 * R * (1.0 + C->gl_r[ir]);
                double wq = wth * 0.5 * R * C->gl_rw[ir] * rho;
                double rv[3], y[3];
                for (int k = 0; k < 3; ++k) { rv[k] = rho * dir[k]; y[k] = xc[k] + rv[k]; }
                cplx U[9], G[27], D1[9], D2[9];
                kernel_U(rv, s, &C->mat, U);
                kernel_gradU(rv, s, &C->mat, G);
                kernel_dU_dc(rv, s, &C->mat, D1, D2);
                vsum += wq * contract(U, w, x, K, L, nrhs, l, j, j);
                gc[0] += wq * creal(contract(D1, w, x, K, L, nrhs, l, j, j));
                gc[1] += wq * creal(contract(D2, w, x, K, L, nrhs, l, j, j));
                for (int k = 0; k < 3; ++k) {
                    cplx Gk[9];
                    for (int q = 0; q < 9; ++q) Gk[q] = G[3 * q + k];
                    double gk = wq * creal(contract(Gk, w, x, K, L, nrhs, l, j, j));
                    for (int b = 0; b < 3; ++b) gv[b][k] += (bary_weight(e, b, y) - 1.0 / 3.0) * gk;
                }
            }
        }
    }
    for (int b = 0; b < 3; ++b)
        for (int k = 0; k < 3; ++k) gv[b][k] += creal(vsum) * dA[b][k] / e->area;
    *val += vsum;
}

/* Value S = sum_{r, l, i, j} w[r][l][i]^T V_ij(s_l) x[r][l][j] of the single layer and the
 * gradient of Re S with respect to the node coordinates and to rho, c_p, c_s: the derivative
 * of the discrete operator, with the pair classes (regular, near level m, self) held fixed.
 * Regular and near pairs: chain rule through the Gauss points y = sum_a beta_a v_a of element
 * j (beta: the 7-point rule's barycentric point mapped into each of the 4^m sub-triangles, so
 * the points move with the vertices), the collocation point (centroid of element i) and the
 * area of element j (each sub-triangle has a 4^-m share of it), with dU/dy from kernel_gradU
 * and dU/dc from kernel_dU_dc.  Self pairs: with fd_h > 0, central differences of the polar
 * rule in each vertex coordinate of the element (step fd_h times its longest edge) and in c_p,
 * c_s (step fd_h times the speed); with fd_h <= 0, the derivative of the integral (self_grad).
 * value: [2]; grad_nodes: [n_nodes][3]; grad_mat: [3] (rho, c_p, c_s). */
int oracle_adjoint_v(const double *nodes, int64_t n_nodes, const int32_t *tris, int64_t K,
                     double rho, double cp, double cs, const double *s, int32_t L, int near_on, double r1,
                     double r2, int self_nt, int self_nr, int32_t nrhs, const double *w, const double *x,
                     double fd_h, double *value, double *grad_nodes, double *grad_mat)
{
    ctx C;
    int rc = setup(&C, nodes, n_nodes, tris, K, rho, cp, cs, near_on, r1, r2, self_nt, self_nr);
    if (rc) return rc;
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    double *gbuf = (double *)calloc((size_t)nth * (3 * (size_t)n_nodes + 5), sizeof(double));
    if (!gbuf) { free((void *)C.el); return -3; }
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *g = gbuf + (size_t)tid * (3 * (size_t)n_nodes + 5);
        double *gm = g + 3 * (size_t)n_nodes;  /* c1, c2, Re S, Im S, (unused) */
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < K; ++i) {
            const element *ei = &C.el[i];
            for (int64_t j = 0; j < K; ++j) {
                const element *ej = &C.el[j];
                const int32_t *tj = tris + 3 * j, *ti = tris + 3 * i;
                if (i == j && fd_h <= 0.0) {
                    double e1v[3], e2v[3], dA[3][3];
                    for (int k = 0; k < 3; ++k) { e1v[k] = ej->v[1][k] - ej->v[0][k]; e2v[k] = ej->v[2][k] - ej->v[0][k]; }
                    const double *n = ej->n;
                    dA[1][0] = 0.5 * (e2v[1] * n[2] - e2v[2] * n[1]);
                    dA[1][1] = 0.5 * (e2v[2] * n[0] - e2v[0] * n[2]);
                    dA[1][2] = 0.5 * (e2v[0] * n[1] - e2v[1] * n[0]);
                    dA[2][0] = 0.5 * (n[1] * e1v[2] - n[2] * e1v[1]);
                    dA[2][1] = 0.5 * (n[2] * e1v[0] - n[0] * e1v[2]);
                    dA[2][2] = 0.5 * (n[0] * e1v[1] - n[1] * e1v[0]);
                    for (int k = 0; k < 3; ++k) dA[0][k] = -(dA[1][k] + dA[2][k]);
                    for (int32_t l = 0; l < L; ++l) {
                        cplx sl = s[2 * l] + I * s[2 * l + 1];
                        cplx v = 0.0;
                        double gv[3][3] = {{0.0}}, gc[2] = {0.0, 0.0};
                        self_grad(&C, ej, sl, w, x, K, L, nrhs, l, j, dA, &v, gv, gc);
                        gm[2] += creal(v);
                        gm[3] += cimag(v);
                        gm[0] += gc[0];
                        gm[1] += gc[1];
                        for (int a = 0; a < 3; ++a)
                            for (int k = 0; k < 3; ++k) g[3 * (int64_t)tj[a] + k] += gv[a][k];
                    }
                    continue;
                }
                if (i == j) {
                    /* value and material derivatives of the self entry, then the vertices */
                    const double hl = fd_h * sqrt(ej->lmax2);
                    for (int32_t l = 0; l < L; ++l) {
                        cplx sl = s[2 * l] + I * s[2 * l + 1];
                        cplx E[9] = {0};
                        self_rule(&C, 0, ej, sl, -1, E);
                        cplx v = contract(E, w, x, K, L, nrhs, l, i, j);
                        gm[2] += creal(v);
                        gm[3] += cimag(v);
                        for (int which = 0; which < 2; ++which) {
                            ctx Cp = C, Cm = C;
                            double h = fd_h * (which == 0 ? cp : cs);
                            if (which == 0) { Cp.mat.c1 += h; Cm.mat.c1 -= h; }
                            else { Cp.mat.c2 += h; Cm.mat.c2 -= h; }
                            cplx Ep[9] = {0}, Em[9] = {0};
                            self_rule(&Cp, 0, ej, sl, -1, Ep);
                            self_rule(&Cm, 0, ej, sl, -1, Em);
                            cplx D[9];
                            for (int t = 0; t < 9; ++t) D[t] = (Ep[t] - Em[t]) / (2.0 * h);
                            gm[which] += creal(contract(D, w, x, K, L, nrhs, l, i, j));
                        }
                        for (int a = 0; a < 3; ++a)
                            for (int k = 0; k < 3; ++k) {
                                double vp[9], vm[9];
                                for (int b = 0; b < 3; ++b)
                                    for (int q = 0; q < 3; ++q) vp[3 * b + q] = vm[3 * b + q] = ej->v[b][q];
                                vp[3 * a + k] += hl;
                                vm[3 * a + k] -= hl;
                                int32_t loc[3] = {0, 1, 2};
                                element ep, em;
                                make_element(vp, loc, &ep);
                                make_element(vm, loc, &em);
                                cplx Ep[9] = {0}, Em[9] = {0};
                                self_rule(&C, 0, &ep, sl, -1, Ep);
                                self_rule(&C, 0, &em, sl, -1, Em);
                                cplx D[9];
                                for (int t = 0; t < 9; ++t) D[t] = (Ep[t] - Em[t]) / (2.0 * hl);
                                g[3 * (int64_t)tj[a] + k] += creal(contract(D, w, x, K, L, nrhs, l, i, j));
                            }
                    }
                    continue;
                }
                /* area derivative of element j: dA/dv1 = (e2 x n)/2, dA/dv2 = (n x e1)/2 */
                double e1v[3], e2v[3], dA[3][3];
                for (int k = 0; k < 3; ++k) { e1v[k] = ej->v[1][k] - ej->v[0][k]; e2v[k] = ej->v[2][k] - ej->v[0][k]; }
                const double *n = ej->n;
                dA[1][0] = 0.5 * (e2v[1] * n[2] - e2v[2] * n[1]);
                dA[1][1] = 0.5 * (e2v[2] * n[0] - e2v[0] * n[2]);
                dA[1][2] = 0.5 * (e2v[0] * n[1] - e2v[1] * n[0]);
                dA[2][0] = 0.5 * (n[1] * e1v[2] - n[2] * e1v[1]);
                dA[2][1] = 0.5 * (n[2] * e1v[0] - n[0] * e1v[2]);
                dA[2][2] = 0.5 * (n[0] * e1v[1] - n[1] * e1v[0]);
                for (int k = 0; k < 3; ++k) dA[0][k] = -(dA[1][k] + dA[2][k]);
                int m = 0;
                if (C.qo.near_on) {
                    double d2 = 0.0;
                    for (int k = 0; k < 3; ++k) d2 += (ei->c[k] - ej->c[k]) * (ei->c[k] - ej->c[k]);
                    if (d2 < C.qo.r1 * C.qo.r1 * ej->lmax2) m = 2;
                    else if (d2 < C.qo.r2 * C.qo.r2 * ej->lmax2) m = 1;
                }
                static const double id[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
                double sub[16][3][3];
                const int nsub = sub_triangles(id[0], id[1], id[2], m, sub, 0);
                for (int qq = 0; qq < 7 * nsub; ++qq) {
                    const int t = qq / 7, q = qq % 7;
                    const double *bq = &C.tri_bary[3 * q];
                    double Bq[3], y[3], rv[3];
                    for (int a = 0; a < 3; ++a) Bq[a] = bq[0] * sub[t][0][a] + bq[1] * sub[t][1][a] + bq[2] * sub[t][2][a];
                    for (int k = 0; k < 3; ++k) {
                        y[k] = Bq[0] * ej->v[0][k] + Bq[1] * ej->v[1][k] + Bq[2] * ej->v[2][k];
                        rv[k] = y[k] - ei->c[k];
                    }
                    const double wq = C.tri_w[q] / nsub, wA = wq * ej->area;
                    for (int32_t l = 0; l < L; ++l) {
                        cplx sl = s[2 * l] + I * s[2 * l + 1];
                        cplx U[9], G[27], D1[9], D2[9];
                        kernel_U(rv, sl, &C.mat, U);
                        kernel_gradU(rv, sl, &C.mat, G);
                        kernel_dU_dc(rv, sl, &C.mat, D1, D2);
                        cplx v = contract(U, w, x, K, L, nrhs, l, i, j);
                        gm[2] += wA * creal(v);
                        gm[3] += wA * cimag(v);
                        gm[0] += wA * creal(contract(D1, w, x, K, L, nrhs, l, i, j));
                        gm[1] += wA * creal(contract(D2, w, x, K, L, nrhs, l, i, j));
                        for (int k = 0; k < 3; ++k) {
                            cplx Gk[9];
                            for (int t = 0; t < 9; ++t) Gk[t] = G[3 * t + k];
                            double gk = wA * creal(contract(Gk, w, x, K, L, nrhs, l, i, j));
                            for (int a = 0; a < 3; ++a) {
                                g[3 * (int64_t)tj[a] + k] += Bq[a] * gk;  /* Gauss point of element j */
                                g[3 * (int64_t)ti[a] + k] -= gk / 3.0;     /* centroid of element i */
                            }
                        }
                        for (int a = 0; a < 3; ++a)
                            for (int k = 0; k < 3; ++k) g[3 * (int64_t)tj[a] + k] += wq * creal(v) * dA[a][k];
                    }
                }
            }
        }
    }
    for (size_t e = 0; e < 3 * (size_t)n_nodes; ++e) grad_nodes[e] = 0.0;
    double gm[4] = {0.0, 0.0, 0.0, 0.0};
    for (int t = 0; t < nth; ++t) {
        const double *g = gbuf + (size_t)t * (3 * (size_t)n_nodes + 5);
        for (size_t e = 0; e < 3 * (size_t)n_nodes; ++e) grad_nodes[e] += g[e];
        for (int k = 0; k < 4; ++k) gm[k] += g[3 * (size_t)n_nodes + k];
    }
    value[0] = gm[2];
    value[1] = gm[3];
    grad_mat[0] = -gm[2] / rho;  /* U is proportional to 1 / rho */
    grad_mat[1] = gm[0];
    grad_mat[2] = gm[1];
    free(gbuf);
    free((void *)C.el);
    return 0;
}

/* Self pair of the double layer differentiated as an integral.  The element stays flat under
 * a perturbation of its vertices; with x = (v_0 + v_1 + v_2) / 3 and y = sum_a lambda_a(y) v_a,
 *   d/dv_a E = PV int d_r T(y - x, n) (lambda_a(y) - 1/3) dy + PV int T(y - x, dn/dv_a) dy
 *              + (dA/dv_a / A) E,
 *   d/dc E = PV int dT/dc dy
 * (T is linear in n, so the second integrand is T with n replaced by dn/dv_a).  Each integrand
 * behaves like G(theta) / rho^2 at x with G odd in the direction: the polar rule of self_rule,
 * per angular line sum_rho w_rho (rho F - G / rho) + G ln R, with G the same integrand for the
 * static kernel (s -> 0, homogeneous of degree -2 in y - x) at unit distance.  Pointwise
 * y-derivatives by central differences of kernel_T (step h |y - x|); the speed derivative as
 * central differences of the rule in c_p, c_s (step h c).  Adds the contraction with w, x at (l, element j): gv[a][k] (Re), gc[2] (Re); dn[a][k]
 * is the derivative of the unit normal with respect to coordinate k of vertex a. */
static void self_grad_k(const ctx *C, const element *e, cplx s, const double *w, const double *x, int64_t K,
                        int32_t L, int32_t nrhs, int32_t l, int64_t j, const double dA[3][3],
                        const double dn[3][3][3], double h, double gv[3][3], double gc[2])
{
    const double *xc = e->c, *n = e->n;
    const cplx s0 = 1e-12;  /* static kernel */
    static const double unit[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
    const double zero[3] = {0.0, 0.0, 0.0};
    double sr[3][3] = {{0.0}}, sn[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < 3; ++a) {
        const double *va = e->v[a], *vb = e->v[(a + 1) % 3];
        double t[3], le = 0.0;
        for (int k = 0; k < 3; ++k) { t[k] = vb[k] - va[k]; le += t[k] * t[k]; }
        le = sqrt(le);
        for (int k = 0; k < 3; ++k) t[k] /= le;
        double proj = 0.0;
        for (int k = 0; k < 3; ++k) proj += (xc[k] - va[k]) * t[k];
        double foot[3], p[3], d = 0.0;
        for (int k = 0; k < 3; ++k) { foot[k] = va[k] + proj * t[k]; p[k] = foot[k] - xc[k]; d += p[k] * p[k]; }
        d = sqrt(d);
        for (int k = 0; k < 3; ++k) p[k] /= d;
        double sa = 0.0, sb = 0.0;
        for (int k = 0; k < 3; ++k) { sa += (va[k] - foot[k]) * t[k]; sb += (vb[k] - foot[k]) * t[k]; }
        double ta = atan2(sa, d), tb = atan2(sb, d);
        for (int it = 0; it < C->qo.self_nt; ++it) {
            double th = 0.5 * (ta + tb) + 0.5 * (tb - ta) * C->gl_t[it];
            double wth = 0.5 * (tb - ta) * C->gl_tw[it];
            double R = d / cos(th);
            double dir[3];
            for (int k = 0; k < 3; ++k) dir[k] = cos(th) * p[k] + sin(th) * t[k];
            /* leading parts at unit distance: the static kernel's y-derivatives and its value
             * with n replaced by e_m */
            double Gr[3], Gn[3], lam1[3];
            for (int b = 0; b < 3; ++b) {
                double y1[3] = {xc[0] + dir[0], xc[1] + dir[1], xc[2] + dir[2]};
                lam1[b] = bary_weight(e, b, y1) - 1.0 / 3.0;  /* (lambda_b - 1/3) per unit distance */
            }
            for (int k = 0; k < 3; ++k) {
                double yp[3] = {dir[0], dir[1], dir[2]}, ym[3] = {dir[0], dir[1], dir[2]};
                yp[k] += h;
                ym[k] -= h;
                cplx Tp[9], Tm[9], D[9];
                kernel_T(zero, yp, n, s0, &C->mat, Tp);
                kernel_T(zero, ym, n, s0, &C->mat, Tm);
                for (int q = 0; q < 9; ++q) D[q] = (Tp[q] - Tm[q]) / (2.0 * h);
                Gr[k] = creal(contract(D, w, x, K, L, nrhs, l, j, j));
                cplx Tn[9];
                kernel_T(zero, dir, unit[k], s0, &C->mat, Tn);
                Gn[k] = creal(contract(Tn, w, x, K, L, nrhs, l, j, j));
            }
            const double lr = log(R);
            for (int k = 0; k < 3; ++k) {
                sn[k] += wth * Gn[k] * lr;
                for (int b = 0; b < 3; ++b) sr[b][k] += wth * Gr[k] * lam1[b] * lr;
            }
            for (int ir = 0; ir < C->qo.self_nr; ++ir) {
                double rho = 0.5 * R * (1.0 + C->gl_r[ir]);
                double wr = 0.5 * R * C->gl_rw[ir];
                double y[3];
                for (int k = 0; k < 3; ++k) y[k] = xc[k] + rho * dir[k];
                const double hy = h * rho;
                for (int k = 0; k < 3; ++k) {
                    double yp[3] = {y[0], y[1], y[2]}, ym[3] = {y[0], y[1], y[2]};
                    yp[k] += hy;
                    ym[k] -= hy;
                    cplx Tp[9], Tm[9], D[9];
                    kernel_T(xc, yp, n, s, &C->mat, Tp);
                    kernel_T(xc, ym, n, s, &C->mat, Tm);
                    for (int q = 0; q < 9; ++q) D[q] = (Tp[q] - Tm[q]) / (2.0 * hy);
                    const double dk = creal(contract(D, w, x, K, L, nrhs, l, j, j));
                    for (int b = 0; b < 3; ++b) {
                        const double lb = bary_weight(e, b, y) - 1.0 / 3.0;
                        sr[b][k] += wth * wr * (rho * dk * lb - Gr[k] * lam1[b] / rho);
                    }
                    cplx Tn[9];
                    kernel_T(xc, y, unit[k], s, &C->mat, Tn);
                    sn[k] += wth * wr * (rho * creal(contract(Tn, w, x, K, L, nrhs, l, j, j)) - Gn[k] / rho);
                }
            }
        }
    }
    /* the value of the self entry for the area term */
    cplx E[9] = {0};
    self_rule(C, 1, e, s, -1, E);
    const double v = creal(contract(E, w, x, K, L, nrhs, l, j, j));
    for (int b = 0; b < 3; ++b)
        for (int k = 0; k < 3; ++k) {
            double g = sr[b][k] + v * dA[b][k] / e->area;
            for (int m = 0; m < 3; ++m) g += dn[b][k][m] * sn[m];
            gv[b][k] += g;
        }
    /* speeds: the rule's points do not move with them, so the central differences of the rule
     * are its integral of dT/dc (with the leading part's derivative) */
    for (int q = 0; q < 2; ++q) {
        ctx Cp = *C, Cm = *C;
        const double hc = h * (q == 0 ? C->mat.c1 : C->mat.c2);
        if (q == 0) { Cp.mat.c1 += hc; Cm.mat.c1 -= hc; }
        else { Cp.mat.c2 += hc; Cm.mat.c2 -= hc; }
        cplx Ep[9] = {0}, Em[9] = {0}, D[9];
        self_rule(&Cp, 1, e, s, -1, Ep);
        self_rule(&Cm, 1, e, s, -1, Em);
        for (int t2 = 0; t2 < 9; ++t2) D[t2] = (Ep[t2] - Em[t2]) / (2.0 * hc);
        gc[q] += creal(contract(D, w, x, K, L, nrhs, l, j, j));
    }
}

/* Value S = sum_{r, l, i, j} w[r][l][i]^T K_ij(s_l) x[r][l][j] of the double layer (op 1; op 2
 * adds the free term I/2, whose derivative is zero) and the gradient of Re S with respect to
 * the node coordinates and c_p, c_s (T does not depend on rho): the derivative of the discrete
 * operator with the pair classes held fixed.  Regular and near pairs: chain rule through the
 * Gauss points of element j (they move with its vertices), its normal n_j = N / |N|,
 * N = (v1 - v0) x (v2 - v0) (dn = (I - n n^T) (dv_a x (v_{a+1} - v_{a+2})) / |N|), its area
 * and the centroid of element i; the pointwise derivatives of T are taken by central
 * differences of kernel_T in y (step fd_h |y - x|) and in c_p, c_s (step fd_h c), and T is
 * linear in n (dT/dn_k = T with n = e_k).  Self pairs: with fd_h > 0, central differences of
 * the polar rule (principal value) in each vertex coordinate (step fd_h times the longest
 * edge) and in the speeds; with fd_h <= 0, the derivative of the integral (self_grad_k), and
 * the pointwise steps are 1e-5.  value: [2]; grad_nodes: [n_nodes][3]; grad_mat: [3] (rho,
 * c_p, c_s). */
int oracle_adjoint_k(const double *nodes, int64_t n_nodes, const int32_t *tris, int64_t K,
                     double rho, double cp, double cs, const double *s, int32_t L, int op, int near_on, double r1,
                     double r2, int self_nt, int self_nr, int32_t nrhs, const double *w, const double *x,
                     double fd_h, double *value, double *grad_nodes, double *grad_mat)
{
    ctx C;
    int rc = setup(&C, nodes, n_nodes, tris, K, rho, cp, cs, near_on, r1, r2, self_nt, self_nr);
    if (rc) return rc;
    const int self_fd = fd_h > 0.0;  /* self pairs by central differences of the rule */
    if (!self_fd) fd_h = 1e-5;
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    double *gbuf = (double *)calloc((size_t)nth * (3 * (size_t)n_nodes + 5), sizeof(double));
    if (!gbuf) { free((void *)C.el); return -3; }
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *g = gbuf + (size_t)tid * (3 * (size_t)n_nodes + 5);
        double *gm = g + 3 * (size_t)n_nodes;
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < K; ++i) {
            const element *ei = &C.el[i];
            for (int64_t j = 0; j < K; ++j) {
                const element *ej = &C.el[j];
                const int32_t *tj = tris + 3 * j, *ti = tris + 3 * i;
                if (i == j && !self_fd) {
                    double e1v[3], e2v[3], dA[3][3], dn[3][3][3];
                    for (int k = 0; k < 3; ++k) { e1v[k] = ej->v[1][k] - ej->v[0][k]; e2v[k] = ej->v[2][k] - ej->v[0][k]; }
                    const double *n = ej->n;
                    dA[1][0] = 0.5 * (e2v[1] * n[2] - e2v[2] * n[1]);
                    dA[1][1] = 0.5 * (e2v[2] * n[0] - e2v[0] * n[2]);
                    dA[1][2] = 0.5 * (e2v[0] * n[1] - e2v[1] * n[0]);
                    dA[2][0] = 0.5 * (n[1] * e1v[2] - n[2] * e1v[1]);
                    dA[2][1] = 0.5 * (n[2] * e1v[0] - n[0] * e1v[2]);
                    dA[2][2] = 0.5 * (n[0] * e1v[1] - n[1] * e1v[0]);
                    for (int k = 0; k < 3; ++k) dA[0][k] = -(dA[1][k] + dA[2][k]);
                    for (int a = 0; a < 3; ++a) {
                        const double *pa1 = ej->v[(a + 1) % 3], *pa2 = ej->v[(a + 2) % 3];
                        double d[3] = {pa1[0] - pa2[0], pa1[1] - pa2[1], pa1[2] - pa2[2]};
                        for (int k = 0; k < 3; ++k) {
                            double ek[3] = {0.0, 0.0, 0.0}, cr[3];
                            ek[k] = 1.0;
                            cr[0] = ek[1] * d[2] - ek[2] * d[1];
                            cr[1] = ek[2] * d[0] - ek[0] * d[2];
                            cr[2] = ek[0] * d[1] - ek[1] * d[0];
                            double nc = n[0] * cr[0] + n[1] * cr[1] + n[2] * cr[2];
                            for (int mm = 0; mm < 3; ++mm) dn[a][k][mm] = (cr[mm] - nc * n[mm]) / (2.0 * ej->area);
                        }
                    }
                    for (int32_t l = 0; l < L; ++l) {
                        cplx sl = s[2 * l] + I * s[2 * l + 1];
                        cplx E[9] = {0};
                        self_rule(&C, 1, ej, sl, -1, E);
                        if (op == 2) { E[0] += 0.5; E[4] += 0.5; E[8] += 0.5; }
                        cplx v = contract(E, w, x, K, L, nrhs, l, i, j);
                        gm[2] += creal(v);
                        gm[3] += cimag(v);
                        double gv[3][3] = {{0.0}}, gc[2] = {0.0, 0.0};
                        self_grad_k(&C, ej, sl, w, x, K, L, nrhs, l, j, dA, dn, fd_h, gv, gc);
                        gm[0] += gc[0];
                        gm[1] += gc[1];
                        for (int a = 0; a < 3; ++a)
                            for (int k = 0; k < 3; ++k) g[3 * (int64_t)tj[a] + k] += gv[a][k];
                    }
                    continue;
                }
                if (i == j) {
                    const double hl = fd_h * sqrt(ej->lmax2);
                    for (int32_t l = 0; l < L; ++l) {
                        cplx sl = s[2 * l] + I * s[2 * l + 1];
                        cplx E[9] = {0};
                        self_rule(&C, 1, ej, sl, -1, E);
                        if (op == 2) { E[0] += 0.5; E[4] += 0.5; E[8] += 0.5; }
                        cplx v = contract(E, w, x, K, L, nrhs, l, i, j);
                        gm[2] += creal(v);
                        gm[3] += cimag(v);
                        for (int which = 0; which < 2; ++which) {
                            ctx Cp = C, Cm = C;
                            double h = fd_h * (which == 0 ? cp : cs);
                            if (which == 0) { Cp.mat.c1 += h; Cm.mat.c1 -= h; }
                            else { Cp.mat.c2 += h; Cm.mat.c2 -= h; }
                            cplx Ep[9] = {0}, Em[9] = {0};
                            self_rule(&Cp, 1, ej, sl, -1, Ep);
                            self_rule(&Cm, 1, ej, sl, -1, Em);
                            cplx D[9];
                            for (int t = 0; t < 9; ++t) D[t] = (Ep[t] - Em[t]) / (2.0 * h);
                            gm[which] += creal(contract(D, w, x, K, L, nrhs, l, i, j));
                        }
                        for (int a = 0; a < 3; ++a)
                            for (int k = 0; k < 3; ++k) {
                                double vp[9], vm[9];
                                for (int b = 0; b < 3; ++b)
                                    for (int q = 0; q < 3; ++q) vp[3 * b + q] = vm[3 * b + q] = ej->v[b][q];
                                vp[3 * a + k] += hl;
                                vm[3 * a + k] -= hl;
                                int32_t loc[3] = {0, 1, 2};
                                element ep, em;
                                make_element(vp, loc, &ep);
                                make_element(vm, loc, &em);
                                cplx Ep[9] = {0}, Em[9] = {0};
                                self_rule(&C, 1, &ep, sl, -1, Ep);
                                self_rule(&C, 1, &em, sl, -1, Em);
                                cplx D[9];
                                for (int t = 0; t < 9; ++t) D[t] = (Ep[t] - Em[t]) / (2.0 * hl);
                                g[3 * (int64_t)tj[a] + k] += creal(contract(D, w, x, K, L, nrhs, l, i, j));
                            }
                    }
                    continue;
                }
                /* area and normal derivatives of element j */
                double e1v[3], e2v[3], dA[3][3], Nn = 0.0;
                for (int k = 0; k < 3; ++k) { e1v[k] = ej->v[1][k] - ej->v[0][k]; e2v[k] = ej->v[2][k] - ej->v[0][k]; }
                const double *n = ej->n;
                dA[1][0] = 0.5 * (e2v[1] * n[2] - e2v[2] * n[1]);
                dA[1][1] = 0.5 * (e2v[2] * n[0] - e2v[0] * n[2]);
                dA[1][2] = 0.5 * (e2v[0] * n[1] - e2v[1] * n[0]);
                dA[2][0] = 0.5 * (n[1] * e1v[2] - n[2] * e1v[1]);
                dA[2][1] = 0.5 * (n[2] * e1v[0] - n[0] * e1v[2]);
                dA[2][2] = 0.5 * (n[0] * e1v[1] - n[1] * e1v[0]);
                for (int k = 0; k < 3; ++k) dA[0][k] = -(dA[1][k] + dA[2][k]);
                Nn = 2.0 * ej->area;
                /* dn[a][k][m]: derivative of n_m with respect to coordinate k of vertex a */
                double dn[3][3][3];
                for (int a = 0; a < 3; ++a) {
                    const double *pa1 = ej->v[(a + 1) % 3], *pa2 = ej->v[(a + 2) % 3];
                    double d[3] = {pa1[0] - pa2[0], pa1[1] - pa2[1], pa1[2] - pa2[2]};
                    for (int k = 0; k < 3; ++k) {
                        double ek[3] = {0.0, 0.0, 0.0}, cr[3];
                        ek[k] = 1.0;
                        cr[0] = ek[1] * d[2] - ek[2] * d[1];
                        cr[1] = ek[2] * d[0] - ek[0] * d[2];
                        cr[2] = ek[0] * d[1] - ek[1] * d[0];
                        double nc = n[0] * cr[0] + n[1] * cr[1] + n[2] * cr[2];
                        for (int mm = 0; mm < 3; ++mm) dn[a][k][mm] = (cr[mm] - nc * n[mm]) / Nn;
                    }
                }
                int m = 0;
                if (C.qo.near_on) {
                    double d2 = 0.0;
                    for (int k = 0; k < 3; ++k) d2 += (ei->c[k] - ej->c[k]) * (ei->c[k] - ej->c[k]);
                    if (d2 < C.qo.r1 * C.qo.r1 * ej->lmax2) m = 2;
                    else if (d2 < C.qo.r2 * C.qo.r2 * ej->lmax2) m = 1;
                }
                static const double id[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
                double sub[16][3][3];
                const int nsub = sub_triangles(id[0], id[1], id[2], m, sub, 0);
                double gn[3] = {0.0, 0.0, 0.0};  /* Re dS/dn_j summed over the points */
                for (int qq = 0; qq < 7 * nsub; ++qq) {
                    const int t = qq / 7, q = qq % 7;
                    const double *bq = &C.tri_bary[3 * q];
                    double Bq[3], y[3];
                    for (int a = 0; a < 3; ++a) Bq[a] = bq[0] * sub[t][0][a] + bq[1] * sub[t][1][a] + bq[2] * sub[t][2][a];
                    double R = 0.0;
                    for (int k = 0; k < 3; ++k) {
                        y[k] = Bq[0] * ej->v[0][k] + Bq[1] * ej->v[1][k] + Bq[2] * ej->v[2][k];
                        R += (y[k] - ei->c[k]) * (y[k] - ei->c[k]);
                    }
                    R = sqrt(R);
                    const double wq = C.tri_w[q] / nsub, wA = wq * ej->area;
                    const double hy = fd_h * R;
                    for (int32_t l = 0; l < L; ++l) {
                        cplx sl = s[2 * l] + I * s[2 * l + 1];
                        cplx T0[9];
                        kernel_T(ei->c, y, n, sl, &C.mat, T0);
                        cplx v = contract(T0, w, x, K, L, nrhs, l, i, j);
                        gm[2] += wA * creal(v);
                        gm[3] += wA * cimag(v);
                        for (int k = 0; k < 3; ++k) {
                            double yp[3] = {y[0], y[1], y[2]}, ym[3] = {y[0], y[1], y[2]};
                            yp[k] += hy;
                            ym[k] -= hy;
                            cplx Tp[9], Tm[9], D[9];
                            kernel_T(ei->c, yp, n, sl, &C.mat, Tp);
                            kernel_T(ei->c, ym, n, sl, &C.mat, Tm);
                            for (int tt = 0; tt < 9; ++tt) D[tt] = (Tp[tt] - Tm[tt]) / (2.0 * hy);
                            double gk = wA * creal(contract(D, w, x, K, L, nrhs, l, i, j));
                            for (int a = 0; a < 3; ++a) {
                                g[3 * (int64_t)tj[a] + k] += Bq[a] * gk;  /* Gauss point of element j */
                                g[3 * (int64_t)ti[a] + k] -= gk / 3.0;     /* centroid of element i */
                            }
                            double ek[3] = {0.0, 0.0, 0.0};
                            ek[k] = 1.0;
                            kernel_T(ei->c, y, ek, sl, &C.mat, D);  /* T is linear in n */
                            gn[k] += wA * creal(contract(D, w, x, K, L, nrhs, l, i, j));
                        }
                        for (int which = 0; which < 2; ++which) {
                            material mp = C.mat, mm_ = C.mat;
                            double h = fd_h * (which == 0 ? cp : cs);
                            if (which == 0) { mp.c1 += h; mm_.c1 -= h; }
                            else { mp.c2 += h; mm_.c2 -= h; }
                            cplx Tp[9], Tm[9], D[9];
                            kernel_T(ei->c, y, n, sl, &mp, Tp);
                            kernel_T(ei->c, y, n, sl, &mm_, Tm);
                            for (int tt = 0; tt < 9; ++tt) D[tt] = (Tp[tt] - Tm[tt]) / (2.0 * h);
                            gm[which] += wA * creal(contract(D, w, x, K, L, nrhs, l, i, j));
                        }
                        for (int a = 0; a < 3; ++a)
                            for (int k = 0; k < 3; ++k) g[3 * (int64_t)tj[a] + k] += wq * creal(v) * dA[a][k];
                    }
                }
                for (int a = 0; a < 3; ++a)
                    for (int k = 0; k < 3; ++k)
                        g[3 * (int64_t)tj[a] + k] += gn[0] * dn[a][k][0] + gn[1] * dn[a][k][1] + gn[2] * dn[a][k][2];
            }
        }
    }
    for (size_t e = 0; e < 3 * (size_t)n_nodes; ++e) grad_nodes[e] = 0.0;
    double gmt[4] = {0.0, 0.0, 0.0, 0.0};
    for (int t = 0; t < nth; ++t) {
        const double *g = gbuf + (size_t)t * (3 * (size_t)n_nodes + 5);
        for (size_t e = 0; e < 3 * (size_t)n_nodes; ++e) grad_nodes[e] += g[e];
        for (int k = 0; k < 4; ++k) gmt[k] += g[3 * (size_t)n_nodes + k];
    }
    value[0] = gmt[2];
    value[1] = gmt[3];
    grad_mat[0] = 0.0;
    grad_mat[1] = gmt[0];
    grad_mat[2] = gmt[1];
    free(gbuf);
    free((void *)C.el);
    return 0;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
