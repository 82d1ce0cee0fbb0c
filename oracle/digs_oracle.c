/*
 * digs_oracle.c -- FP64 CPU oracle of the deformation-informed Gaussian X-ray renderer
 * (DIGS, "Dynamic CBCT Reconstruction using Deformation-Informed 4D Gaussian Splatting and a
 * Low-Rank Free-Form Deformation Model", Huang et al.).
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE. Only the tests, the smoke check and the benchmark's CPU
 * baseline leg may load this library. It shares no code, header, table or helper with the HIP
 * library: it is written from the paper's equations in plain C, in double precision, with no
 * culling, blocking, fusion or reordering beyond what the definitions state.
 *
 * What it computes, in the paper's order:
 *   - Sec. 3.3, Eq. 10: the cubic B-spline free-form deformation u_r(x) of each rank r, on a
 *     uniform control lattice, and (Eq. 11) its spatial Jacobian;
 *   - Sec. 3.3, Eq. 9: the low-rank displacement D(x,t) = x + sum_r w_r(t) u_r(x);
 *   - Sec. 3.2, Eq. 7-8: the deformation-informed warp of each Gaussian, mu' = D(mu),
 *     Sigma' = K Sigma K^T with K = grad D, density unchanged;
 *   - Sec. 3.1, Eq. 2 and the text after it: Sigma = R S S^T R^T, R from a quaternion;
 *   - Sec. 3.1, Eq. 1, 3 and 6: the X-ray transform of the summed Gaussians, i.e. for every
 *     detector pixel the line integral of phi along the ray from the source to the pixel centre.
 *     The integral of one Gaussian along a whole line has the closed form
 *        rho * sqrt(2 pi / a) * exp(-(c - b^2/a)/2),  a = d^T A d, b = d^T A m, c = m^T A m,
 *     with d the unit ray direction, m = source - mu', A = Sigma'^-1. That closed form is the
 *     definition used here, summed over every Gaussian for every pixel (no cut-off);
 *   - the reverse-mode derivative of a scalar loss through all of the above, given dL/dI per
 *     pixel (the objective of Eq. 1), to rho, mu, scale, quaternion, the lattice coefficients and
 *     the temporal weights w_r(t), including the second-derivative (Hessian) term through
 *     K(mu) = I + sum_r w_r grad u_r(mu).
 *
 * Readings of points the paper leaves open (each is listed in the design notes):
 *   - lattice index space is 0-based: control point (i,j,k) sits at origin + (i,j,k)*spacing,
 *     p = (x - origin)/spacing, neighbours floor(p)-1 .. floor(p)+2; indices outside the lattice
 *     are clamped to its edge;
 *   - B_l are the uniform cubic B-spline pieces of the cited Rueckert et al. FFD;
 *   - grad u[a][b] = d u_a / d x_b in world units (divided by the spacing);
 *   - quaternion order (w,x,y,z), normalised inside; scales are linear standard deviations;
 *   - geometry: isocentre at the origin, rotation about z; view angle theta puts the source at
 *     SID (cos t, sin t, 0), the detector centre at (SID - SDD)(cos t, sin t, 0), detector axes
 *     e_u = (-sin t, cos t, 0), e_v = (0,0,1); pixel (row j, column i) centre at
 *     detector centre + (x_i + off_u) e_u + (y_j + off_v) e_v, x_i = (i - (nu-1)/2) pitch_u,
 *     y_j = (j - (nv-1)/2) pitch_v; projections stored proj[t][j][i];
 *   - the projection value is point-sampled at the pixel centre, integrated over the whole line;
 *   - Eq. 4's integration-bias factor (defined in the cited R2-Gaussian work, not in the paper) is
 *     taken as the factor that makes the 2D Gaussian's peak equal the 3D Gaussian's line integral
 *     along the ray through its mean: rho~ = rho sqrt(2 pi / (d^T A d)), d the unit direction of
 *     that ray.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int R, nx, ny, nz;
    double origin[3];
    double spacing[3];
    /* NULL: the motion basis is the lattice's FFD (Eq. 10-11). Otherwise the paper's second
     * ablation (Sec. 4.3): a basis stored per Gaussian, basis[R][12][n] with rows 0..2 the
     * displacement u_{n,r} and rows 3..11 the matrix V_{n,r} (row-major) that replaces grad u_r */
    const double *basis;
} oracle_grid;

typedef struct {
    double sid, sdd;
    int nu, nv;
    double pitch_u, pitch_v, off_u, off_v;
    int model;           /* 0: exact line integral; 1: the 2D-Gaussian approximation of Eq. 4 */
} oracle_geom;

/* ------------------------------------------------------------------------------------------ */
/* Sec. 3.3, Eq. 10: the four pieces of the uniform cubic B-spline, evaluated at the fractional */
/* coordinate u in [0,1), with their first and second derivatives in u.                        */
void oracle_bspline(double u, double B[4], double dB[4], double d2B[4])
{
    double v = 1.0 - u;
    B[0] = v * v * v / 6.0;
    B[1] = (3.0 * u * u * u - 6.0 * u * u + 4.0) / 6.0;
    B[2] = (-3.0 * u * u * u + 3.0 * u * u + 3.0 * u + 1.0) / 6.0;
    B[3] = u * u * u / 6.0;
    dB[0] = -v * v / 2.0;
    dB[1] = (3.0 * u * u - 4.0 * u) / 2.0;
    dB[2] = (-3.0 * u * u + 2.0 * u + 1.0) / 2.0;
    dB[3] = u * u / 2.0;
    d2B[0] = v;
    d2B[1] = 3.0 * u - 2.0;
    d2B[2] = 1.0 - 3.0 * u;
    d2B[3] = u;
}

static int clampi(int i, int n) { return i < 0 ? 0 : (i >= n ? n - 1 : i); }

/* Index of control point (i,j,k) of rank r, component a, in coef[R][nz][ny][nx][3]. */
static size_t coef_index(const oracle_grid *g, int r, int k, int j, int i, int a)
{
    return ((((size_t)r * g->nz + k) * g->ny + j) * g->nx + i) * 3 + a;
}

/* The 4x4x4 stencil of Eq. 10 at point x: for each of the 64 neighbours, its clamped lattice
 * index and its weight, weight gradient (world units) and weight Hessian (world units). */
typedef struct {
    int ii[4], jj[4], kk[4];
    double Bx[4], By[4], Bz[4];
    double dBx[4], dBy[4], dBz[4];
    double d2Bx[4], d2By[4], d2Bz[4];
} stencil;

static void make_stencil(const oracle_grid *g, const double x[3], stencil *s)
{
    double p[3];
    int f[3];
    for (int a = 0; a < 3; ++a) {
        p[a] = (x[a] - g->origin[a]) / g->spacing[a];
        f[a] = (int)floor(p[a]);
    }
    oracle_bspline(p[0] - f[0], s->Bx, s->dBx, s->d2Bx);
    oracle_bspline(p[1] - f[1], s->By, s->dBy, s->d2By);
    oracle_bspline(p[2] - f[2], s->Bz, s->dBz, s->d2Bz);
    for (int l = 0; l < 4; ++l) {
        s->ii[l] = clampi(f[0] - 1 + l, g->nx);
        s->jj[l] = clampi(f[1] - 1 + l, g->ny);
        s->kk[l] = clampi(f[2] - 1 + l, g->nz);
        /* chain rule from lattice index space to world space */
        s->dBx[l] /= g->spacing[0];
        s->dBy[l] /= g->spacing[1];
        s->dBz[l] /= g->spacing[2];
        s->d2Bx[l] /= g->spacing[0] * g->spacing[0];
        s->d2By[l] /= g->spacing[1] * g->spacing[1];
        s->d2Bz[l] /= g->spacing[2] * g->spacing[2];
    }
}

/* weight of stencil point (l,m,n) and its derivatives: w, dw[3], d2w[3][3] */
static void stencil_weight(const stencil *s, int l, int m, int n, double *w, double dw[3],
                           double d2w[3][3])
{
    *w = s->Bx[l] * s->By[m] * s->Bz[n];
    dw[0] = s->dBx[l] * s->By[m] * s->Bz[n];
    dw[1] = s->Bx[l] * s->dBy[m] * s->Bz[n];
    dw[2] = s->Bx[l] * s->By[m] * s->dBz[n];
    if (d2w) {
        d2w[0][0] = s->d2Bx[l] * s->By[m] * s->Bz[n];
        d2w[1][1] = s->Bx[l] * s->d2By[m] * s->Bz[n];
        d2w[2][2] = s->Bx[l] * s->By[m] * s->d2Bz[n];
        d2w[0][1] = d2w[1][0] = s->dBx[l] * s->dBy[m] * s->Bz[n];
        d2w[0][2] = d2w[2][0] = s->dBx[l] * s->By[m] * s->dBz[n];
        d2w[1][2] = d2w[2][1] = s->Bx[l] * s->dBy[m] * s->dBz[n];
    }
}

/* Eq. 10 and Eq. 11 for one rank at one point: u (3), J[a][b] = du_a/dx_b, and optionally the
 * Hessian H[a][b][c] = d^2 u_a / dx_b dx_c. */
static void ffd_point(const oracle_grid *g, const double *coef, int r, const double x[3],
                      double u[3], double J[3][3], double H[3][3][3])
{
    stencil s;
    make_stencil(g, x, &s);
    memset(u, 0, 3 * sizeof(double));
    memset(J, 0, 9 * sizeof(double));
    if (H) memset(H, 0, 27 * sizeof(double));
    for (int n = 0; n < 4; ++n)
        for (int m = 0; m < 4; ++m)
            for (int l = 0; l < 4; ++l) {
                double w, dw[3], d2w[3][3];
                stencil_weight(&s, l, m, n, &w, dw, H ? d2w : NULL);
                for (int a = 0; a < 3; ++a) {
                    double d = coef[coef_index(g, r, s.kk[n], s.jj[m], s.ii[l], a)];
                    u[a] += w * d;
                    for (int b = 0; b < 3; ++b) {
                        J[a][b] += dw[b] * d;
                        if (H)
                            for (int c = 0; c < 3; ++c) H[a][b][c] += d2w[b][c] * d;
                    }
                }
            }
}

/* Public: per-rank FFD value and Jacobian at n points (Eq. 10-11).
 * x[3][n]; U[R][3][n]; V[R][9][n] (row-major 3x3, V[r][3a+b][i] = du_a/dx_b). */
void oracle_ffd_eval(const oracle_grid *g, const double *coef, int n, const double *x, double *U,
                     double *V)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        double xi[3] = {x[i], x[n + i], x[2 * n + i]};
        for (int r = 0; r < g->R; ++r) {
            double u[3], J[3][3];
            ffd_point(g, coef, r, xi, u, J, NULL);
            for (int a = 0; a < 3; ++a) U[((size_t)r * 3 + a) * n + i] = u[a];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) V[((size_t)r * 9 + 3 * a + b) * n + i] = J[a][b];
        }
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Sec. 3.1: rotation from a quaternion (w,x,y,z), normalised first. */
static void quat_rotation(const double q_in[4], double R[3][3], double qh[4], double *qnorm)
{
    double nrm = sqrt(q_in[0] * q_in[0] + q_in[1] * q_in[1] + q_in[2] * q_in[2] + q_in[3] * q_in[3]);
    double w = q_in[0] / nrm, x = q_in[1] / nrm, y = q_in[2] / nrm, z = q_in[3] / nrm;
    R[0][0] = 1 - 2 * (y * y + z * z);
    R[0][1] = 2 * (x * y - w * z);
    R[0][2] = 2 * (x * z + w * y);
    R[1][0] = 2 * (x * y + w * z);
    R[1][1] = 1 - 2 * (x * x + z * z);
    R[1][2] = 2 * (y * z - w * x);
    R[2][0] = 2 * (x * z - w * y);
    R[2][1] = 2 * (y * z + w * x);
    R[2][2] = 1 - 2 * (x * x + y * y);
    if (qh) {
        qh[0] = w; qh[1] = x; qh[2] = y; qh[3] = z;
    }
    if (qnorm) *qnorm = nrm;
}

/* Adjoint of quat_rotation: given dL/dR, dL/dq for the unnormalised q. */
static void quat_rotation_adjoint(const double qh[4], double qnorm, const double gR[3][3],
                                  double gq[4])
{
    double w = qh[0], x = qh[1], y = qh[2], z = qh[3];
    double gw = 0, gx = 0, gy = 0, gz = 0;
    /* R00 = 1 - 2(y^2+z^2) */
    gy += -4 * y * gR[0][0]; gz += -4 * z * gR[0][0];
    /* R01 = 2(xy - wz) */
    gx += 2 * y * gR[0][1]; gy += 2 * x * gR[0][1]; gw += -2 * z * gR[0][1]; gz += -2 * w * gR[0][1];
    /* R02 = 2(xz + wy) */
    gx += 2 * z * gR[0][2]; gz += 2 * x * gR[0][2]; gw += 2 * y * gR[0][2]; gy += 2 * w * gR[0][2];
    /* R10 = 2(xy + wz) */
    gx += 2 * y * gR[1][0]; gy += 2 * x * gR[1][0]; gw += 2 * z * gR[1][0]; gz += 2 * w * gR[1][0];
    /* R11 = 1 - 2(x^2+z^2) */
    gx += -4 * x * gR[1][1]; gz += -4 * z * gR[1][1];
    /* R12 = 2(yz - wx) */
    gy += 2 * z * gR[1][2]; gz += 2 * y * gR[1][2]; gw += -2 * x * gR[1][2]; gx += -2 * w * gR[1][2];
    /* R20 = 2(xz - wy) */
    gx += 2 * z * gR[2][0]; gz += 2 * x * gR[2][0]; gw += -2 * y * gR[2][0]; gy += -2 * w * gR[2][0];
    /* R21 = 2(yz + wx) */
    gy += 2 * z * gR[2][1]; gz += 2 * y * gR[2][1]; gw += 2 * x * gR[2][1]; gx += 2 * w * gR[2][1];
    /* R22 = 1 - 2(x^2+y^2) */
    gx += -4 * x * gR[2][2]; gy += -4 * y * gR[2][2];
    /* through the normalisation qh = q/|q| */
    double gh[4] = {gw, gx, gy, gz};
    double dot = gh[0] * qh[0] + gh[1] * qh[1] + gh[2] * qh[2] + gh[3] * qh[3];
    for (int a = 0; a < 4; ++a) gq[a] = (gh[a] - dot * qh[a]) / qnorm;
}

static void mat_mul(const double A[3][3], const double B[3][3], double C[3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += A[i][k] * B[k][j];
            C[i][j] = s;
        }
}

static void mat_transpose(const double A[3][3], double T[3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) T[i][j] = A[j][i];
}

/* plain 3x3 inverse by cofactors */
static void mat_inverse(const double A[3][3], double Ai[3][3])
{
    double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
    double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
    double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
    double det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
    Ai[0][0] = c00 / det;
    Ai[1][0] = c01 / det;
    Ai[2][0] = c02 / det;
    Ai[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / det;
    Ai[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / det;
    Ai[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / det;
    Ai[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / det;
    Ai[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / det;
    Ai[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / det;
}

/* State of one Gaussian at one time point, after Eq. 7-9. */
typedef struct {
    double mu_t[3];      /* mu' = D(mu, t)                     (Eq. 7, Eq. 9) */
    double K[3][3];      /* K = I + sum_r w_r grad u_r(mu)     (Eq. 11)       */
    double R[3][3];      /* rotation of q                      (Sec. 3.1)     */
    double qh[4], qnorm;
    double S0[3][3];     /* Sigma = R diag(s^2) R^T            (Sec. 3.1)     */
    double St[3][3];     /* Sigma' = K Sigma K^T               (Eq. 8)        */
    double A[3][3];      /* Sigma'^-1                                         */
} gauss_state;

/* rank r of the motion basis at Gaussian k (of n) with canonical mean mu: u_r, grad u_r and (if
 * H is not NULL) its derivative; a per-Gaussian basis does not depend on mu (H = 0) */
static void motion_point(const oracle_grid *g, const double *coef, int r, int k, int n,
                         const double mu[3], double u[3], double J[3][3], double H[3][3][3])
{
    if (!g->basis) {
        ffd_point(g, coef, r, mu, u, J, H);
        return;
    }
    const double *b = g->basis + (size_t)r * 12 * n + k;
    for (int a = 0; a < 3; ++a) {
        u[a] = b[(size_t)a * n];
        for (int c = 0; c < 3; ++c) {
            J[a][c] = b[(size_t)(3 + 3 * a + c) * n];
            if (H)
                for (int e = 0; e < 3; ++e) H[a][c][e] = 0.0;
        }
    }
}

static void deform_one(const oracle_grid *g, const double *coef, int k, int n, const double mu[3],
                       const double s[3], const double q[4], const double *w_t, gauss_state *st)
{
    double K[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    double mt[3] = {mu[0], mu[1], mu[2]};
    for (int r = 0; r < g->R; ++r) {
        double u[3], J[3][3];
        motion_point(g, coef, r, k, n, mu, u, J, NULL);
        for (int a = 0; a < 3; ++a) {
            mt[a] += w_t[r] * u[a];
            for (int b = 0; b < 3; ++b) K[a][b] += w_t[r] * J[a][b];
        }
    }
    memcpy(st->mu_t, mt, sizeof mt);
    memcpy(st->K, K, sizeof K);
    quat_rotation(q, st->R, st->qh, &st->qnorm);
    double D[3][3] = {{s[0] * s[0], 0, 0}, {0, s[1] * s[1], 0}, {0, 0, s[2] * s[2]}};
    double RD[3][3], Rt[3][3], Kt[3][3], KS[3][3];
    mat_mul(st->R, D, RD);
    mat_transpose(st->R, Rt);
    mat_mul(RD, Rt, st->S0);
    mat_mul(K, st->S0, KS);
    mat_transpose(K, Kt);
    mat_mul(KS, Kt, st->St);
    mat_inverse(st->St, st->A);
}

/* Public: Eq. 7-9 for every (t, n). mu_t[T][3][n]; cov_t[T][6][n] packed xx,xy,xz,yy,yz,zz. */
void oracle_deform(const oracle_grid *g, const double *coef, int n, const double *mu,
                   const double *scale, const double *quat, int T, const double *w, double *mu_t,
                   double *cov_t)
{
#pragma omp parallel for schedule(static) collapse(2)
    for (int t = 0; t < T; ++t)
        for (int i = 0; i < n; ++i) {
            double m[3] = {mu[i], mu[n + i], mu[2 * n + i]};
            double s[3] = {scale[i], scale[n + i], scale[2 * n + i]};
            double q[4] = {quat[i], quat[n + i], quat[2 * n + i], quat[3 * n + i]};
            gauss_state st;
            deform_one(g, coef, i, n, m, s, q, w + (size_t)t * g->R, &st);
            for (int a = 0; a < 3; ++a) mu_t[((size_t)t * 3 + a) * n + i] = st.mu_t[a];
            const int pk[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
            for (int c = 0; c < 6; ++c)
                cov_t[((size_t)t * 6 + c) * n + i] = st.St[pk[c][0]][pk[c][1]];
        }
}

/* ------------------------------------------------------------------------------------------ */
/* Cone-beam geometry (reading of the paper's acquisition description, Sec. 4.1). */
static void source_position(const oracle_geom *G, double theta, double s[3])
{
    s[0] = G->sid * cos(theta);
    s[1] = G->sid * sin(theta);
    s[2] = 0.0;
}

static void pixel_centre(const oracle_geom *G, double theta, int j, int i, double P[3])
{
    double ct = cos(theta), sn = sin(theta);
    double cx = (G->sid - G->sdd) * ct, cy = (G->sid - G->sdd) * sn;
    double xu = (i - 0.5 * (G->nu - 1)) * G->pitch_u + G->off_u;
    double yv = (j - 0.5 * (G->nv - 1)) * G->pitch_v + G->off_v;
    P[0] = cx - sn * xu;
    P[1] = cy + ct * xu;
    P[2] = yv;
}

/* Line integral of one Gaussian (Eq. 2) along the whole line through src with unit direction d. */
static double line_integral(const double A[3][3], const double m[3], const double d[3], double rho)
{
    double Ad[3], Am[3];
    for (int a = 0; a < 3; ++a) {
        Ad[a] = A[a][0] * d[0] + A[a][1] * d[1] + A[a][2] * d[2];
        Am[a] = A[a][0] * m[0] + A[a][1] * m[1] + A[a][2] * m[2];
    }
    double aa = d[0] * Ad[0] + d[1] * Ad[1] + d[2] * Ad[2];
    double bb = d[0] * Am[0] + d[1] * Am[1] + d[2] * Am[2];
    double cc = m[0] * Am[0] + m[1] * Am[1] + m[2] * Am[2];
    return rho * sqrt(2.0 * M_PI / aa) * exp(-0.5 * (cc - bb * bb / aa));
}

/* Public: one Gaussian's line integral, given mean, covariance (packed xx,xy,xz,yy,yz,zz),
 * density, a point on the line and a (not necessarily unit) direction. */
double oracle_line_integral(const double mu[3], const double cov6[6], double rho,
                            const double src[3], const double dir[3])
{
    double S[3][3] = {{cov6[0], cov6[1], cov6[2]}, {cov6[1], cov6[3], cov6[4]},
                      {cov6[2], cov6[4], cov6[5]}};
    double A[3][3];
    mat_inverse(S, A);
    double nd = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    double d[3] = {dir[0] / nd, dir[1] / nd, dir[2] / nd};
    double m[3] = {src[0] - mu[0], src[1] - mu[1], src[2] - mu[2]};
    return line_integral(A, m, d, rho);
}

/* ------------------------------------------------------------------------------------------ */
/* Sec. 3.1, Eq. 4: the cone-beam projection of a Gaussian approximated by a 2D Gaussian.
 * The viewing transform W maps world points to the view frame of angle theta (origin at the
 * source; axes e_u, e_v and n, n pointing from the source to the detector centre); the
 * perspective map takes a view-frame point (x, y, z) to detector coordinates SDD (x/z, y/z)
 * (mm, from the detector centre, along e_u and e_v); J is its Jacobian at the mean. The 2D
 * covariance is J W Sigma' W^T J^T (the 2x2 that remains after dropping the third row and
 * column of the 3x3 form), the 2D mean is the image of mu', and the density is scaled by the
 * integration-bias factor (reading in the header). */
typedef struct {
    double m2[2];        /* projected mean (mm on the detector)  */
    double C2[2][2];     /* 2D covariance (mm^2)                 */
    double iC2[2][2];    /* its inverse                          */
    double rho2;         /* rho~                                 */
} ewa_gauss;

static void view_frame(double theta, double W[3][3])
{
    const double ct = cos(theta), sn = sin(theta);
    W[0][0] = -sn; W[0][1] = ct;  W[0][2] = 0.0;    /* e_u */
    W[1][0] = 0.0; W[1][1] = 0.0; W[1][2] = 1.0;    /* e_v */
    W[2][0] = -ct; W[2][1] = -sn; W[2][2] = 0.0;    /* n   */
}

static void ewa_project(const oracle_geom *G, double theta, const double mu_t[3],
                        const double St[3][3], const double A[3][3], double rho, ewa_gauss *e)
{
    double s[3], W[3][3], xv[3] = {0, 0, 0};
    source_position(G, theta, s);
    view_frame(theta, W);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) xv[a] += W[a][b] * (mu_t[b] - s[b]);
    const double x = xv[0], y = xv[1], z = xv[2], f = G->sdd;
    e->m2[0] = f * x / z;
    e->m2[1] = f * y / z;
    /* J (its first two rows) of (x, y, z) -> f (x/z, y/z) */
    const double J[2][3] = {{f / z, 0.0, -f * x / (z * z)}, {0.0, f / z, -f * y / (z * z)}};
    double JW[2][3];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b) {
            JW[a][b] = 0.0;
            for (int k = 0; k < 3; ++k) JW[a][b] += J[a][k] * W[k][b];
        }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            double v = 0.0;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) v += JW[a][k] * St[k][l] * JW[b][l];
            e->C2[a][b] = v;
        }
    const double det = e->C2[0][0] * e->C2[1][1] - e->C2[0][1] * e->C2[1][0];
    e->iC2[0][0] = e->C2[1][1] / det;
    e->iC2[1][1] = e->C2[0][0] / det;
    e->iC2[0][1] = -e->C2[0][1] / det;
    e->iC2[1][0] = -e->C2[1][0] / det;
    /* integration-bias factor: the line integral along the ray through the mean */
    double d[3], nd = 0.0;
    for (int a = 0; a < 3; ++a) {
        d[a] = mu_t[a] - s[a];
        nd += d[a] * d[a];
    }
    nd = sqrt(nd);
    double dAd = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) dAd += (d[a] / nd) * A[a][b] * (d[b] / nd);
    e->rho2 = rho * sqrt(2.0 * M_PI / dAd);
}

static double ewa_value(const ewa_gauss *e, double u, double v)
{
    const double du = u - e->m2[0], dv = v - e->m2[1];
    const double q = du * (e->iC2[0][0] * du + e->iC2[0][1] * dv) +
                     dv * (e->iC2[1][0] * du + e->iC2[1][1] * dv);
    return e->rho2 * exp(-0.5 * q);
}

/* Public: the 2D Gaussian of Eq. 4 for one 3D Gaussian (mean, packed covariance) and view:
 * out[0..1] projected mean, out[2..4] covariance (uu, uv, vv), out[5] rho~. */
void oracle_ewa_gaussian(const oracle_geom *G, double theta, const double mu[3],
                         const double cov6[6], double rho, double out[6])
{
    double S[3][3] = {{cov6[0], cov6[1], cov6[2]}, {cov6[1], cov6[3], cov6[4]},
                      {cov6[2], cov6[4], cov6[5]}};
    double A[3][3];
    mat_inverse(S, A);
    ewa_gauss e;
    ewa_project(G, theta, mu, S, A, rho, &e);
    out[0] = e.m2[0];
    out[1] = e.m2[1];
    out[2] = e.C2[0][0];
    out[3] = e.C2[0][1];
    out[4] = e.C2[1][1];
    out[5] = e.rho2;
}

/* detector coordinates (mm, from the detector centre) of pixel (j, i) */
static void pixel_detector(const oracle_geom *G, int j, int i, double *u, double *v)
{
    *u = (i - 0.5 * (G->nu - 1)) * G->pitch_u + G->off_u;
    *v = (j - 0.5 * (G->nv - 1)) * G->pitch_v + G->off_v;
}

static gauss_state *deform_all(const oracle_grid *g, const double *coef, int n, const double *mu,
                               const double *scale, const double *quat, int T, const double *w)
{
    gauss_state *st = (gauss_state *)malloc(sizeof(gauss_state) * (size_t)T * n);
    if (!st) return NULL;
#pragma omp parallel for schedule(static) collapse(2)
    for (int t = 0; t < T; ++t)
        for (int i = 0; i < n; ++i) {
            double m[3] = {mu[i], mu[n + i], mu[2 * n + i]};
            double s[3] = {scale[i], scale[n + i], scale[2 * n + i]};
            double q[4] = {quat[i], quat[n + i], quat[2 * n + i], quat[3 * n + i]};
            deform_one(g, coef, i, n, m, s, q, w + (size_t)t * g->R, &st[(size_t)t * n + i]);
        }
    return st;
}

/* Eq. 4's 2D Gaussian of every (t, n) */
static ewa_gauss *ewa_all(const oracle_geom *G, const gauss_state *st, int n, const double *rho,
                          int T, const double *angles)
{
    ewa_gauss *e = (ewa_gauss *)malloc(sizeof(ewa_gauss) * (size_t)T * n);
    if (!e) return NULL;
#pragma omp parallel for schedule(static) collapse(2)
    for (int t = 0; t < T; ++t)
        for (int i = 0; i < n; ++i) {
            const gauss_state *gs = &st[(size_t)t * n + i];
            ewa_project(G, angles[t], gs->mu_t, gs->St, gs->A, rho[i], &e[(size_t)t * n + i]);
        }
    return e;
}

/* Public: the forward projection (Eq. 1, 3, 6-9): proj[T][nv][nu] = sum over all Gaussians of
 * the closed-form line integral along the ray from the source to each pixel centre. */
int oracle_project(const oracle_geom *G, const oracle_grid *g, const double *coef, int n,
                   const double *mu, const double *scale, const double *quat, const double *rho,
                   int T, const double *angles, const double *w, double *proj)
{
    gauss_state *st = deform_all(g, coef, n, mu, scale, quat, T, w);
    if (!st) return -1;
    ewa_gauss *ew = NULL;
    if (G->model == 1 && !(ew = ewa_all(G, st, n, rho, T, angles))) {
        free(st);
        return -1;
    }
    const int npx = G->nu * G->nv;
#pragma omp parallel for schedule(dynamic, 16) collapse(2)
    for (int t = 0; t < T; ++t)
        for (int p = 0; p < npx; ++p) {
            int j = p / G->nu, i = p % G->nu;
            if (ew) {
                double u, v, acc = 0.0;
                pixel_detector(G, j, i, &u, &v);
                for (int k = 0; k < n; ++k) acc += ewa_value(&ew[(size_t)t * n + k], u, v);
                proj[(size_t)t * npx + p] = acc;
                continue;
            }
            double s[3], P[3], d[3];
            source_position(G, angles[t], s);
            pixel_centre(G, angles[t], j, i, P);
            double nd = sqrt((P[0] - s[0]) * (P[0] - s[0]) + (P[1] - s[1]) * (P[1] - s[1]) +
                             (P[2] - s[2]) * (P[2] - s[2]));
            for (int a = 0; a < 3; ++a) d[a] = (P[a] - s[a]) / nd;
            double acc = 0.0;
            for (int k = 0; k < n; ++k) {
                const gauss_state *gs = &st[(size_t)t * n + k];
                double m[3] = {s[0] - gs->mu_t[0], s[1] - gs->mu_t[1], s[2] - gs->mu_t[2]};
                acc += line_integral(gs->A, m, d, rho[k]);
            }
            proj[(size_t)t * npx + p] = acc;
        }
    free(ew);
    free(st);
    return 0;
}

/* Public: the same sum at a list of sampled pixels (t, j, i) only. */
int oracle_project_pixels(const oracle_geom *G, const oracle_grid *g, const double *coef, int n,
                          const double *mu, const double *scale, const double *quat,
                          const double *rho, int T, const double *angles, const double *w,
                          int npix, const int *pt, const int *pj, const int *pi, double *out)
{
    gauss_state *st = deform_all(g, coef, n, mu, scale, quat, T, w);
    if (!st) return -1;
    ewa_gauss *ew = NULL;
    if (G->model == 1 && !(ew = ewa_all(G, st, n, rho, T, angles))) {
        free(st);
        return -1;
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int q = 0; q < npix; ++q) {
        int t = pt[q];
        if (ew) {
            double u, v, acc = 0.0;
            pixel_detector(G, pj[q], pi[q], &u, &v);
            for (int k = 0; k < n; ++k) acc += ewa_value(&ew[(size_t)t * n + k], u, v);
            out[q] = acc;
            continue;
        }
        double s[3], P[3], d[3];
        source_position(G, angles[t], s);
        pixel_centre(G, angles[t], pj[q], pi[q], P);
        double nd = sqrt((P[0] - s[0]) * (P[0] - s[0]) + (P[1] - s[1]) * (P[1] - s[1]) +
                         (P[2] - s[2]) * (P[2] - s[2]));
        for (int a = 0; a < 3; ++a) d[a] = (P[a] - s[a]) / nd;
        double acc = 0.0;
        for (int k = 0; k < n; ++k) {
            const gauss_state *gs = &st[(size_t)t * n + k];
            double m[3] = {s[0] - gs->mu_t[0], s[1] - gs->mu_t[1], s[2] - gs->mu_t[2]};
            acc += line_integral(gs->A, m, d, rho[k]);
        }
        out[q] = acc;
    }
    free(ew);
    free(st);
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Reverse mode. Per (t, n): dL/dmu' (3), dL/dK (3x3), dL/dSigma0 (3x3), dL/drho. */
typedef struct {
    double g_mut[3];
    double g_K[3][3];
    double g_S0[3][3];
    double g_rho;
} gauss_grad;

/* Public: gradients of L given dL/dI at a list of pixels (t, j, i, g) -- all other pixels have
 * zero dL/dI. Outputs (overwritten): g_mu[3][n], g_scale[3][n], g_quat[4][n], g_rho[n],
 * g_coef[R][nz][ny][nx][3], g_w[T][R]. */
int oracle_project_bwd(const oracle_geom *G, const oracle_grid *g, const double *coef, int n,
                       const double *mu, const double *scale, const double *quat,
                       const double *rho, int T, const double *angles, const double *w, int npix,
                       const int *pt, const int *pj, const int *pi, const double *pg,
                       double *g_mu, double *g_scale, double *g_quat, double *g_rho,
                       double *g_coef, double *g_w)
{
    if (G->model != 0) return -2;   /* reverse mode of the exact model only */
    gauss_state *st = deform_all(g, coef, n, mu, scale, quat, T, w);
    gauss_grad *gg = (gauss_grad *)calloc((size_t)T * n, sizeof(gauss_grad));
    /* group the pixel entries by projection (order within a projection kept) */
    int *offs = (int *)calloc((size_t)T + 1, sizeof(int));
    int *idx = (int *)malloc(sizeof(int) * (size_t)(npix > 0 ? npix : 1));
    if (!st || !gg || !offs || !idx) {
        free(st);
        free(gg);
        free(offs);
        free(idx);
        return -1;
    }
    for (int q = 0; q < npix; ++q)
        if (pt[q] >= 0 && pt[q] < T) offs[pt[q] + 1]++;
    for (int t = 0; t < T; ++t) offs[t + 1] += offs[t];
    {
        int *fill = (int *)calloc((size_t)T, sizeof(int));
        for (int q = 0; q < npix; ++q)
            if (pt[q] >= 0 && pt[q] < T) idx[offs[pt[q]] + fill[pt[q]]++] = q;
        free(fill);
    }

    /* step 1: through the closed-form line integral to (A, m, rho) and on to (Sigma', mu') */
#pragma omp parallel for schedule(dynamic, 8) collapse(2)
    for (int t = 0; t < T; ++t)
        for (int k = 0; k < n; ++k) {
            const gauss_state *gs = &st[(size_t)t * n + k];
            double s[3];
            source_position(G, angles[t], s);
            double m[3] = {s[0] - gs->mu_t[0], s[1] - gs->mu_t[1], s[2] - gs->mu_t[2]};
            double gA[3][3] = {{0}}, gm[3] = {0}, grho = 0;
            for (int e = offs[t]; e < offs[t + 1]; ++e) {
                int q = idx[e];
                double P[3], d[3];
                pixel_centre(G, angles[t], pj[q], pi[q], P);
                double nd = sqrt((P[0] - s[0]) * (P[0] - s[0]) + (P[1] - s[1]) * (P[1] - s[1]) +
                                 (P[2] - s[2]) * (P[2] - s[2]));
                for (int a = 0; a < 3; ++a) d[a] = (P[a] - s[a]) / nd;
                double Ad[3], Am[3];
                for (int a = 0; a < 3; ++a) {
                    Ad[a] = gs->A[a][0] * d[0] + gs->A[a][1] * d[1] + gs->A[a][2] * d[2];
                    Am[a] = gs->A[a][0] * m[0] + gs->A[a][1] * m[1] + gs->A[a][2] * m[2];
                }
                double aa = d[0] * Ad[0] + d[1] * Ad[1] + d[2] * Ad[2];
                double bb = d[0] * Am[0] + d[1] * Am[1] + d[2] * Am[2];
                double cc = m[0] * Am[0] + m[1] * Am[1] + m[2] * Am[2];
                double base = sqrt(2.0 * M_PI / aa) * exp(-0.5 * (cc - bb * bb / aa));
                double val = rho[k] * base;
                double gv = pg[q];
                grho += gv * base;
                double ga = gv * val * (-0.5 / aa - 0.5 * bb * bb / (aa * aa));
                double gb = gv * val * (bb / aa);
                double gc = gv * val * (-0.5);
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b)
                        gA[a][b] += ga * d[a] * d[b] + gb * d[a] * m[b] + gc * m[a] * m[b];
                for (int a = 0; a < 3; ++a) {
                    /* b = d^T A m -> db/dm = A^T d; c = m^T A m -> dc/dm = (A + A^T) m */
                    double Atd = gs->A[0][a] * d[0] + gs->A[1][a] * d[1] + gs->A[2][a] * d[2];
                    double Atm = gs->A[0][a] * m[0] + gs->A[1][a] * m[1] + gs->A[2][a] * m[2];
                    gm[a] += gb * Atd + gc * (Am[a] + Atm);
                }
            }
            gauss_grad *out = &gg[(size_t)t * n + k];
            out->g_rho = grho;
            /* m = s - mu' */
            for (int a = 0; a < 3; ++a) out->g_mut[a] = -gm[a];
            /* A = Sigma'^-1: dL/dSigma' = -A^T gA A^T */
            double At[3][3], tmp[3][3], gSt[3][3];
            mat_transpose(gs->A, At);
            mat_mul(At, gA, tmp);
            mat_mul(tmp, At, gSt);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) gSt[a][b] = -gSt[a][b];
            /* Sigma' = K Sigma0 K^T: dL/dK = gSt K Sigma0^T + gSt^T K Sigma0,
             * dL/dSigma0 = K^T gSt K */
            double KS0[3][3], KS0t[3][3], S0t[3][3], gStT[3][3], Kt[3][3], a1[3][3], a2[3][3];
            mat_transpose(gs->S0, S0t);
            mat_mul(gs->K, S0t, KS0t);
            mat_mul(gs->K, gs->S0, KS0);
            mat_transpose(gSt, gStT);
            mat_mul(gSt, KS0t, a1);
            mat_mul(gStT, KS0, a2);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) out->g_K[a][b] = a1[a][b] + a2[a][b];
            mat_transpose(gs->K, Kt);
            mat_mul(Kt, gSt, tmp);
            mat_mul(tmp, gs->K, out->g_S0);
        }

    /* step 2: through Sigma0 = R diag(s^2) R^T, the quaternion, and D(mu,t) of Eq. 9-11 */
    if (!g->basis) memset(g_coef, 0, sizeof(double) * (size_t)g->R * g->nz * g->ny * g->nx * 3);
    memset(g_w, 0, sizeof(double) * (size_t)T * g->R);
    for (int k = 0; k < n; ++k) {
        double m0[3] = {mu[k], mu[n + k], mu[2 * n + k]};
        double s[3] = {scale[k], scale[n + k], scale[2 * n + k]};
        double q[4] = {quat[k], quat[n + k], quat[2 * n + k], quat[3 * n + k]};
        double R[3][3], qh[4], qn;
        quat_rotation(q, R, qh, &qn);
        double gS0[3][3] = {{0}}, gmu[3] = {0}, grho = 0;
        double P[8][3], Q[8][3][3]; /* sum_t w_r(t) dL/dmu', sum_t w_r(t) dL/dK */
        memset(P, 0, sizeof P);
        memset(Q, 0, sizeof Q);
        double U[8][3], J[8][3][3], H[8][3][3][3];
        for (int r = 0; r < g->R; ++r) motion_point(g, coef, r, k, n, m0, U[r], J[r], H[r]);
        for (int t = 0; t < T; ++t) {
            const gauss_grad *gr = &gg[(size_t)t * n + k];
            const double *wt = w + (size_t)t * g->R;
            grho += gr->g_rho;
            for (int a = 0; a < 3; ++a) {
                gmu[a] += gr->g_mut[a];
                for (int b = 0; b < 3; ++b) gS0[a][b] += gr->g_S0[a][b];
            }
            for (int r = 0; r < g->R; ++r) {
                double gw = 0;
                for (int a = 0; a < 3; ++a) {
                    gw += gr->g_mut[a] * U[r][a];
                    P[r][a] += wt[r] * gr->g_mut[a];
                    for (int b = 0; b < 3; ++b) {
                        gw += gr->g_K[a][b] * J[r][a][b];
                        Q[r][a][b] += wt[r] * gr->g_K[a][b];
                    }
                }
                g_w[(size_t)t * g->R + r] += gw;
            }
        }
        /* mu' = mu + sum_r w_r u_r(mu); K = I + sum_r w_r grad u_r(mu) (a per-Gaussian basis
         * does not depend on mu: mu' - mu and K carry no further mu-dependence) */
        for (int r = 0; r < g->R && !g->basis; ++r)
            for (int c = 0; c < 3; ++c)
                for (int a = 0; a < 3; ++a) {
                    gmu[c] += J[r][a][c] * P[r][a];
                    for (int b = 0; b < 3; ++b) gmu[c] += Q[r][a][b] * H[r][a][b][c];
                }
        if (g->basis) {   /* dL/du_{n,r} = P_r, dL/dV_{n,r} = Q_r (written into g_coef) */
            for (int r = 0; r < g->R; ++r)
                for (int a = 0; a < 3; ++a) {
                    g_coef[((size_t)r * 12 + a) * n + k] = P[r][a];
                    for (int b = 0; b < 3; ++b)
                        g_coef[((size_t)r * 12 + 3 + 3 * a + b) * n + k] = Q[r][a][b];
                }
        }
        /* coefficients: u_r and grad u_r are linear in d^r */
        stencil sc;
        if (!g->basis) make_stencil(g, m0, &sc);
        for (int nn = 0; nn < 4 && !g->basis; ++nn)
            for (int mm = 0; mm < 4; ++mm)
                for (int l = 0; l < 4; ++l) {
                    double wt, dw[3];
                    stencil_weight(&sc, l, mm, nn, &wt, dw, NULL);
                    for (int r = 0; r < g->R; ++r)
                        for (int a = 0; a < 3; ++a) {
                            double v = wt * P[r][a];
                            for (int b = 0; b < 3; ++b) v += dw[b] * Q[r][a][b];
                            g_coef[coef_index(g, r, sc.kk[nn], sc.jj[mm], sc.ii[l], a)] += v;
                        }
                }
        /* Sigma0 = R D R^T, D = diag(s^2) */
        double D[3][3] = {{s[0] * s[0], 0, 0}, {0, s[1] * s[1], 0}, {0, 0, s[2] * s[2]}};
        double gS0t[3][3], sumg[3][3], RD[3][3], gR[3][3], Rt[3][3], tmp[3][3], RtgR[3][3];
        mat_transpose(gS0, gS0t);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) sumg[a][b] = gS0[a][b] + gS0t[a][b];
        mat_mul(R, D, RD);
        mat_mul(sumg, RD, gR);
        mat_transpose(R, Rt);
        mat_mul(Rt, gS0, tmp);
        mat_mul(tmp, R, RtgR);
        double gq[4];
        quat_rotation_adjoint(qh, qn, gR, gq);
        for (int a = 0; a < 3; ++a) {
            g_mu[(size_t)a * n + k] = gmu[a];
            g_scale[(size_t)a * n + k] = 2.0 * s[a] * RtgR[a][a];
        }
        for (int a = 0; a < 4; ++a) g_quat[(size_t)a * n + k] = gq[a];
        g_rho[k] = grho;
    }
    free(st);
    free(gg);
    free(offs);
    free(idx);
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Eq. 6 and Eq. 9 on a set of query points: the displacement sum_r w_r u_r(x) (DVF) and the
 * dynamic attenuation phi(x,t) = sum_n rho_n exp(-(x - mu')^T Sigma'^-1 (x - mu')/2). */
void oracle_dvf(const oracle_grid *g, const double *coef, const double *w_t, int npts,
                const double *x, double *dvf)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < npts; ++i) {
        double xi[3] = {x[i], x[npts + i], x[2 * npts + i]};
        double acc[3] = {0, 0, 0};
        for (int r = 0; r < g->R; ++r) {
            double u[3], J[3][3];
            ffd_point(g, coef, r, xi, u, J, NULL);
            for (int a = 0; a < 3; ++a) acc[a] += w_t[r] * u[a];
        }
        for (int a = 0; a < 3; ++a) dvf[(size_t)a * npts + i] = acc[a];
    }
}

void oracle_phi(int n, const double *mu_t, const double *cov_t, const double *rho, int npts,
                const double *x, double *phi)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < npts; ++i) {
        double acc = 0;
        for (int k = 0; k < n; ++k) {
            double S[3][3] = {{cov_t[k], cov_t[n + k], cov_t[2 * n + k]},
                              {cov_t[n + k], cov_t[3 * n + k], cov_t[4 * n + k]},
                              {cov_t[2 * n + k], cov_t[4 * n + k], cov_t[5 * n + k]}};
            double A[3][3];
            mat_inverse(S, A);
            double dx[3] = {x[i] - mu_t[k], x[npts + i] - mu_t[n + k], x[2 * npts + i] - mu_t[2 * n + k]};
            double qf = 0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) qf += dx[a] * A[a][b] * dx[b];
            acc += rho[k] * exp(-0.5 * qf);
        }
        phi[i] = acc;
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Sec. 3.3 (text after Eq. 11) and Sec. 4.2: the temporal weights w_r(t) of the low-rank motion
 * model are a 1-D cubic B-spline in time over control values c[j][r] placed every `dt` (the paper
 * uses a control point every 4 time points) starting at t0. The same 0-based knot and clamping
 * convention as the spatial lattice: p = (t - t0)/dt, f = floor(p), u = p - f,
 * w_r(t) = sum_l B_l(u) c[clamp(f - 1 + l)][r]. */
void oracle_temporal_weights(int Ct, int R, const double *ctrl, double t0, double dt, int T,
                             const double *times, double *w)
{
    for (int t = 0; t < T; ++t) {
        double p = (times[t] - t0) / dt, f = floor(p), B[4], dB[4], d2B[4];
        oracle_bspline(p - f, B, dB, d2B);
        for (int r = 0; r < R; ++r) {
            double acc = 0.0;
            for (int l = 0; l < 4; ++l) acc += B[l] * ctrl[(size_t)clampi((int)f - 1 + l, Ct) * R + r];
            w[(size_t)t * R + r] = acc;
        }
    }
}

/* Reverse mode of the above: g_ctrl[j][r] = sum over t and l with clamp(f_t - 1 + l) = j of
 * B_l(u_t) g_w[t][r]. */
void oracle_temporal_weights_bwd(int Ct, int R, double t0, double dt, int T, const double *times,
                                 const double *g_w, double *g_ctrl)
{
    memset(g_ctrl, 0, sizeof(double) * (size_t)Ct * R);
    for (int t = 0; t < T; ++t) {
        double p = (times[t] - t0) / dt, f = floor(p), B[4], dB[4], d2B[4];
        oracle_bspline(p - f, B, dB, d2B);
        for (int l = 0; l < 4; ++l)
            for (int r = 0; r < R; ++r)
                g_ctrl[(size_t)clampi((int)f - 1 + l, Ct) * R + r] += B[l] * g_w[(size_t)t * R + r];
    }
}
