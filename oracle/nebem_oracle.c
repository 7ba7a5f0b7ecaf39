/*
 * nebem_oracle.c -- plain, slow, FP64 CPU oracle for the neBEM hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no source with the HIP path.
 *
 * What it computes (paper, "Numerical Formulation" and Sec. 2.1):
 *   Phi'(P) = integral over the panel S of dA / |P - s|            (potential kernel)
 *   E'(P)   = integral over S of (P - s) / |P - s|^3 dA            (field kernel)
 * for a uniformly charged flat rectangle or right triangle; the physical
 * potential/field of density sigma are k_e*sigma*Phi' and k_e*sigma*E' with
 * k_e = 1/(4 pi eps0) (Green's function of the Laplace operator, Eq. Green).
 *
 * How: near the panel (R < 8 D, R = distance to the centroid, D = panel
 * diameter) the exact integral is written as a sum over the polygon's edges
 * (the standard closed form for a uniform density on a planar polygon:
 * D. R. Wilton et al., IEEE Trans. Antennas Propag. 32(3):276-281, 1984;
 * R. D. Graglia, IEEE TAP 41(10):1448-1455, 1993).  Far from it (R >= 8 D)
 * the integrand is smooth and an 8x8 Gauss-Legendre rule (collapsed onto the
 * triangle for right triangles) reaches the integral to rounding.
 *
 * Then, following the paper: influence matrix by collocation at centroids
 * (Eq. Matrix, K rho = phi), potential/field at arbitrary points by
 * superposition over elements and their periodic copies (Eqs. Potential,
 * Field; "virtual copies" of the base cell, Sec. 3 and Sec. 5.2), and the
 * point-charge sums of the space-charge algorithm (Sec. 4.2, Algorithm 2),
 * generalised to the field and to every charge as a target.
 *
 * Readings where the paper is silent (normal convention, on-panel principal
 * value, dielectric interface rows, mirror copies) are stated at the
 * functions that apply them.
 *
 * Sums are accumulated with Neumaier's compensated summation in a fixed order
 * (panels in index order, copies in lattice order).  OpenMP only splits the
 * independent outer loop (points / rows).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define EPS0 8.8541878128e-12 /* vacuum permittivity, F/m (CODATA 2018) */
static const double KE = 1.0 / (4.0 * 3.14159265358979323846 * EPS0);

/* ---------------------------------------------------------------- vectors */
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double *a) { return sqrt(dot3(a, a)); }
static void sub3(const double *a, const double *b, double *c)
{
    c[0] = a[0] - b[0];
    c[1] = a[1] - b[1];
    c[2] = a[2] - b[2];
}

/* Neumaier compensated accumulator */
typedef struct { double s, c; } acc_t;
static void acc_add(acc_t *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static double acc_get(const acc_t *a) { return a->s + a->c; }

/* ----------------------------------------------------- Gauss-Legendre rule */
#define GL_M 8
static double gl_x[GL_M], gl_w[GL_M]; /* nodes/weights on [0,1] */
static int gl_ready = 0;

/* Nodes are the roots of the Legendre polynomial P_m, found by Newton's
 * method from the usual cosine starting guesses; weights 2/((1-x^2) P_m'(x)^2).
 * Mapped from [-1,1] to [0,1]. */
static void gl_init(void)
{
    if (gl_ready) return;
    for (int i = 0; i < GL_M; ++i) {
        double x = cos(3.14159265358979323846 * (i + 0.75) / (GL_M + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= GL_M; ++k) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = GL_M * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-17) break;
        }
        {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= GL_M; ++k) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = GL_M * (x * p1 - p0) / (x * x - 1.0);
        }
        gl_x[i] = 0.5 * (1.0 - x);
        gl_w[i] = 1.0 / ((1.0 - x * x) * dp * dp); /* = 0.5 * 2/((1-x^2)P'^2) */
    }
    gl_ready = 1;
}

/* ------------------------------------------------------ panel description */
/* kind 0: rectangle o + s u + t w (0 <= s,t <= 1)
 * kind 1: right triangle o + s u + t w (s,t >= 0, s + t <= 1)
 * Vertices listed counter-clockwise about n = u x w / |u x w|. */
static int panel_vertices(int kind, const double *o, const double *u, const double *w, double V[4][3])
{
    for (int k = 0; k < 3; ++k) {
        V[0][k] = o[k];
        V[1][k] = o[k] + u[k];
        if (kind == 0) {
            V[2][k] = o[k] + u[k] + w[k];
            V[3][k] = o[k] + w[k];
        } else {
            V[2][k] = o[k] + w[k];
        }
    }
    return kind == 0 ? 4 : 3;
}

/* ln((R+ + l+)/(R- + l-)) for one edge, written so that no difference of
 * nearly equal numbers is formed:
 *  - if l+ + l- < 0 the edge is traversed backwards (uses (R+l)(R-l) = R0^2);
 *  - (R+ + l+)/(R- + l-) - 1 = L (R+ + R- + l+ + l-)/((R+ + R-)(R- + l-)),
 *    from R+ - R- = (l+^2 - l-^2)/(R+ + R-) and l+ - l- = L;
 *  - R- + l- = R0^2/(R- - l-) when l- < 0. */
static double edge_log(double lp, double lm, double Rp, double Rm, double R0sq, double L)
{
    if (lp + lm < 0.0) {
        double t = lp;
        lp = -lm;
        lm = -t;
        t = Rp;
        Rp = Rm;
        Rm = t;
    }
    double S = Rp + Rm + lp + lm;
    double den = (lm >= 0.0) ? (Rm + lm) : R0sq / (Rm - lm);
    return log1p(L * S / ((Rp + Rm) * den));
}

/* Exact Phi', E' of a planar polygon at P (edge formula).  If on_plane is set
 * the height above the panel plane is taken as exactly 0: the observation
 * point is the panel's own collocation point and the normal field takes its
 * principal value 0 (the average of the two one-sided limits +-2 pi). */
static void polygon_exact(int nv, double V[4][3], const double *nrm, const double *P, int on_plane, double out[4])
{
    double dtrue = (P[0] - V[0][0]) * nrm[0] + (P[1] - V[0][1]) * nrm[1] + (P[2] - V[0][2]) * nrm[2];
    double rho[3] = {P[0] - dtrue * nrm[0], P[1] - dtrue * nrm[1], P[2] - dtrue * nrm[2]};
    double d = on_plane ? 0.0 : dtrue;
    double ad = fabs(d);
    double R[4];
    for (int k = 0; k < nv; ++k) {
        double r[3];
        sub3(on_plane ? rho : P, V[k], r);
        R[k] = norm3(r);
    }
    acc_t phi = {0, 0}, om = {0, 0}, ex = {0, 0}, ey = {0, 0}, ez = {0, 0};
    for (int k = 0; k < nv; ++k) {
        const double *A = V[k], *B = V[(k + 1) % nv];
        double e[3], t[3], m[3], ar[3], br[3];
        sub3(B, A, e);
        double L = norm3(e);
        for (int i = 0; i < 3; ++i) t[i] = e[i] / L;
        cross3(t, nrm, m); /* outward in-plane edge normal */
        sub3(A, rho, ar);
        sub3(B, rho, br);
        double P0 = dot3(ar, m);
        double lm = dot3(ar, t), lp = dot3(br, t);
        double Rm = R[k], Rp = R[(k + 1) % nv];
        double R0sq = P0 * P0 + d * d;
        double lam = edge_log(lp, lm, Rp, Rm, R0sq, L);
        double beta = atan2(P0 * lp, R0sq + ad * Rp) - atan2(P0 * lm, R0sq + ad * Rm);
        acc_add(&phi, P0 == 0.0 ? 0.0 : P0 * lam);
        acc_add(&om, beta);
        acc_add(&ex, m[0] * lam);
        acc_add(&ey, m[1] * lam);
        acc_add(&ez, m[2] * lam);
    }
    double omega = acc_get(&om);
    double sg = (d > 0.0) ? 1.0 : (d < 0.0 ? -1.0 : 0.0);
    out[0] = acc_get(&phi) - ad * omega;
    out[1] = acc_get(&ex) + sg * omega * nrm[0];
    out[2] = acc_get(&ey) + sg * omega * nrm[1];
    out[3] = acc_get(&ez) + sg * omega * nrm[2];
}

/* Far field: Gauss-Legendre quadrature of the smooth integrand. */
static void panel_gauss(int kind, const double *o, const double *u, const double *w, const double *P, double out[4])
{
    double uw[3];
    cross3(u, w, uw);
    double jac = norm3(uw);
    acc_t a[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    for (int i = 0; i < GL_M; ++i)
        for (int j = 0; j < GL_M; ++j) {
            double s, t, wt;
            if (kind == 0) {
                s = gl_x[i];
                t = gl_x[j];
                wt = gl_w[i] * gl_w[j];
            } else { /* collapsed map (xi, eta) -> (xi, (1 - xi) eta) onto s + t <= 1 */
                s = gl_x[i];
                t = (1.0 - gl_x[i]) * gl_x[j];
                wt = gl_w[i] * gl_w[j] * (1.0 - gl_x[i]);
            }
            double r[3];
            for (int k = 0; k < 3; ++k) r[k] = P[k] - (o[k] + s * u[k] + t * w[k]);
            double rr = norm3(r);
            double inv = 1.0 / rr, inv3 = inv * inv * inv;
            acc_add(&a[0], wt * inv);
            acc_add(&a[1], wt * r[0] * inv3);
            acc_add(&a[2], wt * r[1] * inv3);
            acc_add(&a[3], wt * r[2] * inv3);
        }
    for (int k = 0; k < 4; ++k) out[k] = jac * acc_get(&a[k]);
}

/* Phi', E' of one panel at P.  Near/far threshold R/D = 8. */
void oracle_panel(int kind, const double *o, const double *u, const double *w, const double *P, int on_plane,
                  double *out)
{
    gl_init();
    double V[4][3], nrm[3], c[3], dvec[3];
    int nv = panel_vertices(kind, o, u, w, V);
    cross3(u, w, nrm);
    double nn = norm3(nrm);
    for (int k = 0; k < 3; ++k) nrm[k] /= nn;
    double f = (kind == 0) ? 0.5 : (1.0 / 3.0);
    for (int k = 0; k < 3; ++k) c[k] = o[k] + f * (u[k] + w[k]);
    double diag[3];
    for (int k = 0; k < 3; ++k) diag[k] = (kind == 0) ? (u[k] + w[k]) : (u[k] - w[k]);
    double D = norm3(diag);
    sub3(P, c, dvec);
    double R = norm3(dvec);
    if (!on_plane && R >= 8.0 * D)
        panel_gauss(kind, o, u, w, P, out);
    else
        polygon_exact(nv, V, nrm, P, on_plane, out);
}

/* Exact-only variant (edge formula at every distance), for the pins. */
void oracle_panel_exact(int kind, const double *o, const double *u, const double *w, const double *P, int on_plane,
                        double *out)
{
    double V[4][3], nrm[3];
    int nv = panel_vertices(kind, o, u, w, V);
    cross3(u, w, nrm);
    double nn = norm3(nrm);
    for (int k = 0; k < 3; ++k) nrm[k] /= nn;
    polygon_exact(nv, V, nrm, P, on_plane, out);
}

/* Quadrature-only variant with the 8x8 rule, for the pins. */
void oracle_panel_gauss(int kind, const double *o, const double *u, const double *w, const double *P, double *out)
{
    gl_init();
    panel_gauss(kind, o, u, w, P, out);
}

/* ---------------------------------------------------------------- images */
/* Copies of the base cell: translations t = n1 a1 + n2 a2 (|n1| <= N1,
 * |n2| <= N2; n1 outer loop) combined with every subset of the reflection
 * planes x_k = mpos[k] selected by mask; a copy reflected in a set of planes
 * carries the product of their parities.  copy = t + M(panel), so its
 * kernel at P is M applied to the base panel's kernel at M(P - t).
 * (Periodic copies: paper Sec. 3 and Sec. 5.2; mirror copies are a reading,
 * the paper does not describe them.) */
typedef struct {
    double a1[3], a2[3];
    int32_t n1, n2;
    int32_t mirror_mask;
    double mirror_pos[3];
    int32_t mirror_parity[3];
} oracle_images;

static int n_reflections(const oracle_images *im) { return 1 << __builtin_popcount(im->mirror_mask & 7); }

/* r-th subset of the active reflection axes, as an axis bit mask */
static int reflection_axes(const oracle_images *im, int r)
{
    int axes = 0, bit = 0;
    for (int k = 0; k < 3; ++k)
        if (im->mirror_mask & (1 << k)) {
            if (r & (1 << bit)) axes |= (1 << k);
            ++bit;
        }
    return axes;
}

/* accumulates parity * M(kernel(M(P - t))) for every copy of one panel */
static void panel_all_copies(int kind, const double *o, const double *u, const double *w, const oracle_images *im,
                             const double *P, int self_index_copy, double out[4])
{
    acc_t a[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    int nr = n_reflections(im);
    for (int r = 0; r < nr; ++r) {
        int axes = reflection_axes(im, r);
        double par = 1.0;
        for (int k = 0; k < 3; ++k)
            if (axes & (1 << k)) par *= (double)im->mirror_parity[k];
        for (int i = -im->n1; i <= im->n1; ++i)
            for (int j = -im->n2; j <= im->n2; ++j) {
                double Q[3], v[4];
                for (int k = 0; k < 3; ++k) {
                    Q[k] = P[k] - (i * im->a1[k] + j * im->a2[k]);
                    if (axes & (1 << k)) Q[k] = 2.0 * im->mirror_pos[k] - Q[k];
                }
                int on_plane = self_index_copy && r == 0 && i == 0 && j == 0;
                oracle_panel(kind, o, u, w, Q, on_plane, v);
                for (int k = 0; k < 3; ++k)
                    if (axes & (1 << k)) v[1 + k] = -v[1 + k];
                for (int k = 0; k < 4; ++k) acc_add(&a[k], par * v[k]);
            }
    }
    for (int k = 0; k < 4; ++k) out[k] = acc_get(&a[k]);
}

/* ------------------------------------------------------------------ eval */
/* phi(P) = k_e sum_j sigma_j sum_copies Phi'_j, E likewise (Eqs. Potential
 * and Field with a uniform density per element).  pts, out row-major:
 * pts[m][3], out[m][4] = (phi, Ex, Ey, Ez). */
void oracle_eval(int64_t n, const int32_t *kind, const double *o, const double *u, const double *w,
                 const double *sigma, const oracle_images *im, int64_t m, const double *pts, double *out, int nthreads)
{
    gl_init();
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (int64_t p = 0; p < m; ++p) {
        acc_t a[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
        for (int64_t j = 0; j < n; ++j) {
            double v[4];
            panel_all_copies(kind[j], o + 3 * j, u + 3 * j, w + 3 * j, im, pts + 3 * p, 0, v);
            for (int k = 0; k < 4; ++k) acc_add(&a[k], sigma[j] * v[k]);
        }
        for (int k = 0; k < 4; ++k) out[4 * p + k] = KE * acc_get(&a[k]);
    }
}

/* -------------------------------------------------------------- assembly */
/* Influence matrix by collocation (Eq. Matrix), column-major A[i + j*n]:
 *  conductor row i:  A_ij = k_e sum_copies Phi'_j(c_i)
 *  dielectric row i: A_ij = k_e sum_copies n_i . E'_j(c_i)
 *                           + delta_ij (eps+ + eps-)/(2 eps0 (eps+ - eps-))
 * The dielectric row is continuity of the normal displacement across an
 * interface carrying a total (free + polarisation) single-layer density in
 * vacuum -- a reading: the paper restricts its formulation to Dirichlet
 * conditions.  With E_pv the principal-value field at c_i and the two
 * one-sided fields E_pv +- sigma_i/(2 eps0) n_i:
 *   eps+ (E_pv.n + sigma_i/2eps0) = eps- (E_pv.n - sigma_i/2eps0).
 * Collocation points: colloc (n x 3) or, if NULL, the panel centroids.  Row i
 * treats its own panel (identity copy) as lying exactly in its plane. */
/* Rows `rows[0..nrows)` of the influence matrix, out[r][j] row-major
 * (nrows x n).  Same definitions as oracle_assemble. */
void oracle_assemble_rows(int64_t n, const int32_t *kind, const double *o, const double *u, const double *w,
                          const int32_t *bc, const double *eps_pos, const double *eps_neg, const oracle_images *im,
                          const double *colloc, int64_t nrows, const int64_t *rows, double *out, int nthreads)
{
    gl_init();
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (int64_t rr = 0; rr < nrows; ++rr) {
        const int64_t i = rows[rr];
        double ci[3], ni[3];
        double f = (kind[i] == 0) ? 0.5 : (1.0 / 3.0);
        for (int k = 0; k < 3; ++k)
            ci[k] = colloc ? colloc[3 * i + k] : o[3 * i + k] + f * (u[3 * i + k] + w[3 * i + k]);
        cross3(u + 3 * i, w + 3 * i, ni);
        double nn = norm3(ni);
        for (int k = 0; k < 3; ++k) ni[k] /= nn;
        for (int64_t j = 0; j < n; ++j) {
            double v[4];
            panel_all_copies(kind[j], o + 3 * j, u + 3 * j, w + 3 * j, im, ci, i == j, v);
            double a;
            if (bc[i] == 0) {
                a = KE * v[0];
            } else {
                a = KE * (ni[0] * v[1] + ni[1] * v[2] + ni[2] * v[3]);
                if (i == j) a += (eps_pos[i] + eps_neg[i]) / (2.0 * EPS0 * (eps_pos[i] - eps_neg[i]));
            }
            out[rr * n + j] = a;
        }
    }
}

/* Whole influence matrix, column-major A[i + j*n]. */
void oracle_assemble(int64_t n, const int32_t *kind, const double *o, const double *u, const double *w,
                     const int32_t *bc, const double *eps_pos, const double *eps_neg, const oracle_images *im,
                     const double *colloc, double *A, int nthreads)
{
    double *rowbuf = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
    int64_t *rows = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) rows[i] = i;
    oracle_assemble_rows(n, kind, o, u, w, bc, eps_pos, eps_neg, im, colloc, n, rows, rowbuf, nthreads);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) A[i + j * n] = rowbuf[i * n + j];
    free(rowbuf);
    free(rows);
}

/* ------------------------------------------------------- point charges */
/* phi, E at nt targets from ns point charges (Algorithm 2's sum, also for
 * the field): k_e sum_j q_j / r and k_e sum_j q_j (x - x_j)/r^3, skipping
 * the target's own index (self[t] = j, or -1) and any source at distance 0.
 * out[nt][4]. */
void oracle_coulomb(int64_t nt, const double *tgt, const int64_t *self, int64_t ns, const double *src,
                    const double *q, double *out, double *absum, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (int64_t t = 0; t < nt; ++t) {
        acc_t a[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
        acc_t m = {0, 0};
        int64_t me = self ? self[t] : -1;
        for (int64_t j = 0; j < ns; ++j) {
            if (j == me) continue;
            double r[3];
            sub3(tgt + 3 * t, src + 3 * j, r);
            double r2 = dot3(r, r);
            if (r2 == 0.0) continue;
            double rr = sqrt(r2);
            double inv = 1.0 / rr, inv3 = inv / r2;
            acc_add(&a[0], q[j] * inv);
            acc_add(&a[1], q[j] * r[0] * inv3);
            acc_add(&a[2], q[j] * r[1] * inv3);
            acc_add(&a[3], q[j] * r[2] * inv3);
            acc_add(&m, fabs(q[j]) / r2);
        }
        for (int k = 0; k < 4; ++k) out[4 * t + k] = KE * acc_get(&a[k]);
        if (absum) absum[t] = KE * acc_get(&m);
    }
}

double oracle_ke(void) { return KE; }
double oracle_eps0(void) { return EPS0; }
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
