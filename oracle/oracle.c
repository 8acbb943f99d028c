/*
 * Plain FP64 CPU oracle for the partial-assembly Lagrange-phase operators.
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the package's smoke check and the
 * benchmark's CPU-baseline leg may load this library. It shares no code,
 * header, table or constant with the GPU library.
 *
 * What it computes (paper: "Matrix-free approaches for GPU acceleration of a
 * high-order finite element hydrodynamics application", Sec. 2.1 and Sec. 3):
 *
 *   semi-discrete Lagrange system (Sec. 3.3, eqs. semiDiscreteLagStart..End)
 *       M_v dv/dt = -F 1,   M_E de/dt = F^T v,   dx/dt = v,
 *       rho |J| = rho0 |J0|                       (pointwise mass conservation)
 *   with the total stress = ideal-gas pressure + artificial viscosity (Sec. 2.1).
 *
 * Every operator is evaluated by its plain definition: 3-D basis functions are
 * evaluated directly at each quadrature point (products of 1-D Lagrange
 * values), dense element matrices are formed, and they are applied element by
 * element with a fixed-order scatter. There is no sum factorisation here; the
 * paper states the partially assembled operators give the same results as the
 * fully assembled ones (Sec. 6), which is what the GPU path is checked against.
 *
 * Readings of what the paper leaves open (all stated again in the design doc):
 *   - reference element [0,1]^3; H1 = Q_p nodal Lagrange at Gauss-Lobatto
 *     points; L2 = Q_{p-1} nodal Lagrange at the Gauss-Legendre points of a
 *     p-point rule; quadrature = tensor Gauss-Legendre with Q points per axis;
 *   - force matrix F[(i,c), j] = int sigma : grad(w_i e_c) phi_j dx, the
 *     bilinear form behind M_v dv/dt = -F 1 and M_E de/dt = F^T v;
 *   - ideal gas p = (gamma-1) rho e, c_s = sqrt(gamma (gamma-1) max(e,0));
 *   - scalar viscosity mu = rho l (q1 c_s + q2 l max(0, -tr eps)),
 *     l = detJ^(1/3)/p, sigma = -p I + mu eps, eps = sym(grad v);
 *   - rho = rho0 detJ0 / detJ, so m_q = rho0 detJ0 w_q is time independent.
 *
 * Functions with "absmode" != 0 run the same loops on absolute values of every
 * factor; that gives the sum of magnitudes of all terms, the natural scale for
 * rounding-error comparisons.
 *
 * Arithmetic rules: elements ascending, local DOFs ascending, quadrature
 * points lexicographic; built with -O2 -ffp-contract=off, no fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXP 8
#define OR_MAXQ 12

/* ------------------------------------------------------------------ 1-D rules */

/* Legendre polynomial P_n(s) and its derivative, by the three-term recurrence. */
static double legendre(int n, double s, double *dP)
{
    double p0 = 1.0, p1 = s;
    if (n == 0) { *dP = 0.0; return 1.0; }
    for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * s * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    /* (1 - s^2) P_n' = n (P_{n-1} - s P_n) */
    *dP = n * (p0 - s * p1) / (1.0 - s * s);
    return p1;
}

/* Gauss-Legendre rule with n points on [0,1] (Sec. 3.4 names the standard
 * Gauss-Legendre rule): Newton on P_n(s), s = 2t - 1, from Chebyshev-like
 * guesses; weight 1 / ((1 - s^2) P_n'(s)^2) on [0,1]. Points ascend. */
int or_gauss_legendre(int n, double *t, double *w)
{
    if (n < 1 || n > OR_MAXQ) return -1;
    for (int k = 0; k < n; ++k) {
        double s = -cos(M_PI * (k + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double dP, P = legendre(n, s, &dP);
            double ds = P / dP;
            s -= ds;
            if (fabs(ds) < 1e-17) break;
        }
        double dP;
        legendre(n, s, &dP);
        t[k] = 0.5 * (s + 1.0);
        w[k] = 1.0 / ((1.0 - s * s) * dP * dP);
    }
    return 0;
}

/* Gauss-Lobatto points (p+1 of them) on [0,1]: 0, 1 and the roots of P_p'.
 * Newton on P_p' with P_p'' from Legendre's equation
 * (1 - s^2) P'' = 2 s P' - p (p+1) P. */
int or_gll_nodes(int p, double *t)
{
    if (p < 1 || p > OR_MAXP - 1) return -1;
    t[0] = 0.0;
    t[p] = 1.0;
    for (int k = 1; k < p; ++k) {
        double s = -cos(M_PI * k / p);
        for (int it = 0; it < 100; ++it) {
            double dP, P = legendre(p, s, &dP);
            double d2P = (2.0 * s * dP - p * (p + 1.0) * P) / (1.0 - s * s);
            double ds = dP / d2P;
            s -= ds;
            if (fabs(ds) < 1e-17) break;
        }
        t[k] = 0.5 * (s + 1.0);
    }
    return 0;
}

/* Lagrange basis of the nodes t[0..n-1] at x: values l_a(x) and derivatives. */
void or_lagrange(int n, const double *t, double x, double *val, double *der)
{
    for (int a = 0; a < n; ++a) {
        double v = 1.0;
        for (int b = 0; b < n; ++b)
            if (b != a) v *= (x - t[b]) / (t[a] - t[b]);
        val[a] = v;
        double d = 0.0;
        for (int m = 0; m < n; ++m) {
            if (m == a) continue;
            double term = 1.0 / (t[a] - t[m]);
            for (int b = 0; b < n; ++b)
                if (b != a && b != m) term *= (x - t[b]) / (t[a] - t[b]);
            d += term;
        }
        der[a] = d;
    }
}

/* L2 nodes of Q_{p-1}: the p Gauss-Legendre points. */
static void l2_nodes(int p, double *t)
{
    double w[OR_MAXQ];
    or_gauss_legendre(p, t, w);
}

/* -------------------------------------------------------- per-element basis */

/* 1-D tables at the quadrature points: H1 values/derivatives, L2 values. */
typedef struct {
    int p, D, Dl, Q;
    double tq[OR_MAXQ], wq[OR_MAXQ];
    double hv[OR_MAXQ][OR_MAXP], hd[OR_MAXQ][OR_MAXP]; /* [q][a] */
    double lv[OR_MAXQ][OR_MAXP];                      /* [q][b] */
} or_basis;

static int make_basis(int p, int Q, or_basis *bs)
{
    if (p < 1 || p + 1 > OR_MAXP || Q < 1 || Q > OR_MAXQ) return -1;
    double th[OR_MAXP], tl[OR_MAXP], dummy[OR_MAXP];
    bs->p = p;
    bs->D = p + 1;
    bs->Dl = p;
    bs->Q = Q;
    or_gauss_legendre(Q, bs->tq, bs->wq);
    or_gll_nodes(p, th);
    l2_nodes(p, tl);
    for (int q = 0; q < Q; ++q) {
        or_lagrange(p + 1, th, bs->tq[q], bs->hv[q], bs->hd[q]);
        or_lagrange(p, tl, bs->tq[q], bs->lv[q], dummy);
    }
    return 0;
}

/* 3-D H1 basis value and reference gradient of local node i at qp (qx,qy,qz). */
static void h1_at(const or_basis *bs, int i, int qx, int qy, int qz, double *val, double grad[3])
{
    int D = bs->D;
    int ix = i % D, iy = (i / D) % D, iz = i / (D * D);
    double vx = bs->hv[qx][ix], vy = bs->hv[qy][iy], vz = bs->hv[qz][iz];
    double dx = bs->hd[qx][ix], dy = bs->hd[qy][iy], dz = bs->hd[qz][iz];
    *val = vx * vy * vz;
    grad[0] = dx * vy * vz;
    grad[1] = vx * dy * vz;
    grad[2] = vx * vy * dz;
}

/* 3-D L2 basis value of local node j at qp (qx,qy,qz). */
static double l2_at(const or_basis *bs, int j, int qx, int qy, int qz)
{
    int Dl = bs->Dl;
    int jx = j % Dl, jy = (j / Dl) % Dl, jz = j / (Dl * Dl);
    return bs->lv[qx][jx] * bs->lv[qy][jy] * bs->lv[qz][jz];
}

static double det3(const double A[3][3])
{
    return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1])
         - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0])
         + A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}

/* inverse by the adjugate: inv = adj(A) / det(A) */
static void inv3(const double A[3][3], double det, double inv[3][3])
{
    inv[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / det;
    inv[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / det;
    inv[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / det;
    inv[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / det;
    inv[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / det;
    inv[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / det;
    inv[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / det;
    inv[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / det;
    inv[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / det;
}

/* element list helper: elems == NULL means all elements */
#define ELEM(k) (elems ? elems[k] : (int32_t)(k))
#define NLOOP (elems ? n_sel : n_elem)

/* --------------------------------------------------------------- qdata */

/*
 * Quadrature data of every (selected) element, Sec. 3.1's "D" of the force and
 * mass operators:
 *   S[e][c][d][q] = w_q detJ_q sum_k sigma_q[c][k] Jinv_q[d][k]  (w detJ sigma J^-T)
 *   mq[e][q]      = rho0 detJ0_q w_q                             (rho |J| = rho0 |J0|)
 *                   (or_qdata_pt: rho0_q[e][q] detJ0_q w_q, an initial density
 *                   given at every point, when rho0_q != NULL)
 *   detJ[e][q]    (optional)
 *   dt[e][q]      (optional) the stable explicit time step of the point: the
 *                 time a signal of speed c_s + mu/(rho l) needs to cross the
 *                 length l = detJ^(1/3)/p, i.e. l / ((1+q1) c_s + q2 l max(0, -tr eps))
 *                 (+inf where both speeds vanish); a reading, the paper names
 *                 no time-step rule
 * Inputs: x0, x, v as [3][N]; e as [E][p^3]. Any output pointer may be NULL.
 * Returns 0, or -1 on bad arguments, or -2 when some detJ <= 0 (values still
 * written).
 */
int or_qdata_pt(int n_elem, int p, int Q, int N, const int32_t *map,
                const double *x0, const double *x, const double *v, const double *e,
                double rho0, const double *rho0_q, double gamma, double q1, double q2,
                const int32_t *elems, int n_sel,
                double *S, double *mq, double *detJ_out, double *dt_out)
{
    or_basis bs;
    if (make_basis(p, Q, &bs)) return -1;
    const int D = bs.D, D3 = D * D * D, Dl3 = p * p * p, Q3 = Q * Q * Q;
    int bad = 0;
    for (int k = 0; k < NLOOP; ++k) {
        const int el = ELEM(k);
        const int32_t *nodes = map + (size_t)el * D3;
        for (int qz = 0; qz < Q; ++qz)
        for (int qy = 0; qy < Q; ++qy)
        for (int qx = 0; qx < Q; ++qx) {
            const int q = qx + Q * (qy + Q * qz);
            const double w = bs.wq[qx] * bs.wq[qy] * bs.wq[qz];
            double J[3][3] = {{0}}, J0[3][3] = {{0}}, Gv[3][3] = {{0}};
            for (int i = 0; i < D3; ++i) {
                double val, g[3];
                h1_at(&bs, i, qx, qy, qz, &val, g);
                const int32_t gi = nodes[i];
                for (int c = 0; c < 3; ++c)
                    for (int d = 0; d < 3; ++d) {
                        J[c][d] += x[(size_t)c * N + gi] * g[d];
                        J0[c][d] += x0[(size_t)c * N + gi] * g[d];
                        if (v) Gv[c][d] += v[(size_t)c * N + gi] * g[d];
                    }
            }
            const double dJ = det3(J), dJ0 = det3(J0);
            if (!(dJ > 0.0)) bad = 1;
            const double r0 = rho0_q ? rho0_q[(size_t)el * Q3 + q] : rho0;
            const double m = r0 * dJ0 * w;
            if (mq) mq[(size_t)el * Q3 + q] = m;
            if (detJ_out) detJ_out[(size_t)el * Q3 + q] = dJ;
            if (!S && !dt_out) continue;
            double Ji[3][3];
            inv3(J, dJ, Ji);
            const double rho = m / (w * dJ);
            double eq = 0.0;
            if (e)
                for (int j = 0; j < Dl3; ++j)
                    eq += e[(size_t)el * Dl3 + j] * l2_at(&bs, j, qx, qy, qz);
            const double pres = (gamma - 1.0) * rho * eq;
            const double cs = sqrt(gamma * (gamma - 1.0) * (eq > 0.0 ? eq : 0.0));
            /* physical velocity gradient grad v = (ref gradient) J^-1 */
            double L[3][3];
            for (int c = 0; c < 3; ++c)
                for (int kk = 0; kk < 3; ++kk) {
                    double s = 0.0;
                    for (int d = 0; d < 3; ++d) s += Gv[c][d] * Ji[d][kk];
                    L[c][kk] = s;
                }
            double eps[3][3];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) eps[a][b] = 0.5 * (L[a][b] + L[b][a]);
            const double tr = eps[0][0] + eps[1][1] + eps[2][2];
            const double ell = cbrt(dJ) / p;
            const double mu = rho * ell * (q1 * cs + q2 * ell * (tr < 0.0 ? -tr : 0.0));
            if (dt_out) {
                const double speed = cs + mu / (rho * ell);
                dt_out[(size_t)el * Q3 + q] = speed > 0.0 ? ell / speed : INFINITY;
            }
            if (!S) continue;
            double sig[3][3];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) sig[a][b] = mu * eps[a][b] - (a == b ? pres : 0.0);
            for (int c = 0; c < 3; ++c)
                for (int d = 0; d < 3; ++d) {
                    double s = 0.0;
                    for (int kk = 0; kk < 3; ++kk) s += sig[c][kk] * Ji[d][kk];
                    S[(((size_t)el * 3 + c) * 3 + d) * Q3 + q] = w * dJ * s;
                }
        }
    }
    return bad ? -2 : 0;
}

int or_qdata(int n_elem, int p, int Q, int N, const int32_t *map,
             const double *x0, const double *x, const double *v, const double *e,
             double rho0, double gamma, double q1, double q2,
             const int32_t *elems, int n_sel,
             double *S, double *mq, double *detJ_out, double *dt_out)
{
    return or_qdata_pt(n_elem, p, Q, N, map, x0, x, v, e, rho0, NULL, gamma, q1, q2, elems, n_sel,
                       S, mq, detJ_out, dt_out);
}

/* ------------------------------------------------------- multi-material */

/*
 * Quadrature data of the multi-material force operators F_k (Sec. 2.1's
 * multi-material momentum and energy equations, rho dv/dt = div sum_k eta_k
 * sigma_k and eta_k rho_k de_k/dt = eta_k sigma_k : grad v; Sec. 3.3's
 * semi-discrete M_v dv/dt = -sum_k F_k 1, M_E,k de_k/dt = F_k^T v - c_k,
 * eta_k rho_k |J| = eta_k0 rho_k0 |J0|), for K materials:
 *   F_k[(i,c), j] = int eta_k sigma_k : grad(w_i e_c) phi_j dx
 *   S_k[e][c][d][q] = w_q detJ_q sum_m (eta_k sigma_k)[c][m] Jinv[d][m]
 * Readings: no closure model (alpha_k = 0, c_k = 0), so eta_k = eta_k0 along
 * the motion and rho_k = rho_k0 detJ0/detJ; eta_k0 is an L2 field (the
 * thermodynamic space, like e_k) with coefficients eta0[k][e][j];
 * sigma_k = -p_k I + mu_k eps with p_k = (gamma_k - 1) rho_k e_k and the
 * scalar viscosity mu_k = rho_k l (q1 c_s,k + q2 l max(0, -tr eps)),
 * c_s,k = sqrt(gamma_k (gamma_k - 1) max(e_k, 0)), l = detJ^(1/3)/p.
 * Also mqk[k][e][q] = eta_k0 rho_k0 detJ0 w (the material's mass per point)
 * when mqk != NULL. Inputs e[k][e][j], eta0[k][e][j] ([K][E][p^3]),
 * gamma[k], rho0[k]. Returns 0, -1 on bad arguments, -2 if some detJ <= 0.
 */
int or_qdata_mm(int n_elem, int p, int Q, int N, const int32_t *map, int K,
                const double *x0, const double *x, const double *v, const double *e,
                const double *eta0, const double *gamma, const double *rho0, double q1, double q2,
                double *S, double *mqk)
{
    or_basis bs;
    if (make_basis(p, Q, &bs) || K < 1) return -1;
    const int D = bs.D, D3 = D * D * D, Dl3 = p * p * p, Q3 = Q * Q * Q;
    const size_t Sk = (size_t)n_elem * 9 * Q3, Mk = (size_t)n_elem * Q3, Lk = (size_t)n_elem * Dl3;
    int bad = 0;
    for (int el = 0; el < n_elem; ++el) {
        const int32_t *nodes = map + (size_t)el * D3;
        for (int qz = 0; qz < Q; ++qz)
        for (int qy = 0; qy < Q; ++qy)
        for (int qx = 0; qx < Q; ++qx) {
            const int q = qx + Q * (qy + Q * qz);
            const double w = bs.wq[qx] * bs.wq[qy] * bs.wq[qz];
            double J[3][3] = {{0}}, J0[3][3] = {{0}}, Gv[3][3] = {{0}};
            for (int i = 0; i < D3; ++i) {
                double val, g[3];
                h1_at(&bs, i, qx, qy, qz, &val, g);
                for (int c = 0; c < 3; ++c)
                    for (int d = 0; d < 3; ++d) {
                        J[c][d] += x[(size_t)c * N + nodes[i]] * g[d];
                        J0[c][d] += x0[(size_t)c * N + nodes[i]] * g[d];
                        Gv[c][d] += v[(size_t)c * N + nodes[i]] * g[d];
                    }
            }
            const double dJ = det3(J), dJ0 = det3(J0);
            if (!(dJ > 0.0)) bad = 1;
            double Ji[3][3];
            inv3(J, dJ, Ji);
            double L[3][3];
            for (int c = 0; c < 3; ++c)
                for (int m = 0; m < 3; ++m) {
                    double s = 0.0;
                    for (int d = 0; d < 3; ++d) s += Gv[c][d] * Ji[d][m];
                    L[c][m] = s;
                }
            double eps[3][3];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) eps[a][b] = 0.5 * (L[a][b] + L[b][a]);
            const double tr = eps[0][0] + eps[1][1] + eps[2][2];
            const double ell = cbrt(dJ) / p;
            for (int k = 0; k < K; ++k) {
                double eta = 0.0, ek = 0.0;
                for (int j = 0; j < Dl3; ++j) {
                    const double phi = l2_at(&bs, j, qx, qy, qz);
                    eta += eta0[k * Lk + (size_t)el * Dl3 + j] * phi;
                    ek += e[k * Lk + (size_t)el * Dl3 + j] * phi;
                }
                const double rho = rho0[k] * dJ0 / dJ;  /* eta_k rho_k |J| = eta_k0 rho_k0 |J0| */
                const double pk = (gamma[k] - 1.0) * rho * ek;
                const double cs = sqrt(gamma[k] * (gamma[k] - 1.0) * (ek > 0.0 ? ek : 0.0));
                const double mu = rho * ell * (q1 * cs + q2 * ell * (tr < 0.0 ? -tr : 0.0));
                if (mqk) mqk[k * Mk + (size_t)el * Q3 + q] = eta * rho0[k] * dJ0 * w;
                for (int c = 0; c < 3; ++c)
                    for (int d = 0; d < 3; ++d) {
                        double s = 0.0;
                        for (int m = 0; m < 3; ++m) {
                            const double sig = mu * eps[c][m] - (c == m ? pk : 0.0);
                            s += eta * sig * Ji[d][m];
                        }
                        S[k * Sk + (((size_t)el * 3 + c) * 3 + d) * Q3 + q] = w * dJ * s;
                    }
            }
        }
    }
    return bad ? -2 : 0;
}

/* -------------------------------------------------------- element matrices */

/* 3-D basis tables at every quadrature point, evaluated directly as products of
 * 1-D values: hv3[q][i], hg3[q][i][d] (reference gradient), lv3[q][j]. */
typedef struct {
    int Q3, D3, Dl3;
    double *hv3, *hg3, *lv3;
} or_tab3;

static int make_tab3(const or_basis *bs, or_tab3 *tb)
{
    const int Q = bs->Q, D3 = bs->D * bs->D * bs->D, Dl3 = bs->Dl * bs->Dl * bs->Dl;
    tb->Q3 = Q * Q * Q;
    tb->D3 = D3;
    tb->Dl3 = Dl3;
    tb->hv3 = (double *)malloc(sizeof(double) * tb->Q3 * D3);
    tb->hg3 = (double *)malloc(sizeof(double) * tb->Q3 * D3 * 3);
    tb->lv3 = (double *)malloc(sizeof(double) * tb->Q3 * Dl3);
    if (!tb->hv3 || !tb->hg3 || !tb->lv3) return -3;
    for (int qz = 0; qz < Q; ++qz)
    for (int qy = 0; qy < Q; ++qy)
    for (int qx = 0; qx < Q; ++qx) {
        const int q = qx + Q * (qy + Q * qz);
        for (int i = 0; i < D3; ++i)
            h1_at(bs, i, qx, qy, qz, &tb->hv3[q * D3 + i], &tb->hg3[(q * D3 + i) * 3]);
        for (int j = 0; j < Dl3; ++j) tb->lv3[q * Dl3 + j] = l2_at(bs, j, qx, qy, qz);
    }
    return 0;
}

static void free_tab3(or_tab3 *tb)
{
    free(tb->hv3);
    free(tb->hg3);
    free(tb->lv3);
}

/*
 * Dense element force matrix of one element from its quadrature data:
 *   FE[(c*D^3 + i) * Dl^3 + j] = sum_q sum_d S[c][d](q) dw_i/dxi_d(q) phi_j(q).
 * Every entry sums its terms with q lexicographic outer and d inner.
 */
static void force_elem(const or_tab3 *tb, const double *S_el, int absmode, double *FE)
{
    const int D3 = tb->D3, Dl3 = tb->Dl3, Q3 = tb->Q3;
    memset(FE, 0, sizeof(double) * 3 * D3 * Dl3);
    for (int q = 0; q < Q3; ++q)
        for (int c = 0; c < 3; ++c)
            for (int i = 0; i < D3; ++i) {
                const double *g = &tb->hg3[(q * D3 + i) * 3];
                for (int j = 0; j < Dl3; ++j) {
                    const double phi = tb->lv3[q * Dl3 + j];
                    double *acc = &FE[(c * D3 + i) * Dl3 + j];
                    for (int d = 0; d < 3; ++d) {
                        const double s = S_el[(c * 3 + d) * Q3 + q];
                        if (absmode) *acc += fabs(s) * fabs(g[d]) * fabs(phi);
                        else *acc += s * g[d] * phi;
                    }
                }
            }
}

/* Element mass matrix ME[i*D^3 + j] = sum_q m_q w_i(q) w_j(q) (Sec. 3.2's M_E). */
static void mass_elem(const or_tab3 *tb, const double *mq_el, int absmode, double *ME)
{
    const int D3 = tb->D3, Q3 = tb->Q3;
    memset(ME, 0, sizeof(double) * D3 * D3);
    for (int q = 0; q < Q3; ++q) {
        const double m = mq_el[q];
        for (int i = 0; i < D3; ++i) {
            const double vi = tb->hv3[q * D3 + i];
            for (int j = 0; j < D3; ++j) {
                const double vj = tb->hv3[q * D3 + j];
                ME[i * D3 + j] += absmode ? fabs(m) * fabs(vi) * fabs(vj) : m * vi * vj;
            }
        }
    }
}

/*
 * Thermodynamic (L2) mass matrix of every element, the M_E of the energy
 * equation M_E de/dt = F^T v (Sec. 3.3): ME[e][j][k] = sum_q rho_q detJ_q w_q
 * phi_j(q) phi_k(q), and rho detJ w = m_q by rho |J| = rho0 |J0|, so M_E does
 * not change while the mesh moves. phi are evaluated directly at each point.
 */
int or_l2_mass(int n_elem, int p, int Q, const double *mq, double *ME)
{
    or_basis bs;
    if (make_basis(p, Q, &bs)) return -1;
    const int Dl3 = p * p * p, Q3 = Q * Q * Q;
    for (int el = 0; el < n_elem; ++el) {
        double *M = ME + (size_t)el * Dl3 * Dl3;
        memset(M, 0, sizeof(double) * Dl3 * Dl3);
        for (int qz = 0; qz < Q; ++qz)
        for (int qy = 0; qy < Q; ++qy)
        for (int qx = 0; qx < Q; ++qx) {
            const int q = qx + Q * (qy + Q * qz);
            const double m = mq[(size_t)el * Q3 + q];
            for (int j = 0; j < Dl3; ++j) {
                const double pj = l2_at(&bs, j, qx, qy, qz);
                for (int k = 0; k < Dl3; ++k) M[j * Dl3 + k] += m * pj * l2_at(&bs, k, qx, qy, qz);
            }
        }
    }
    return 0;
}

/* Export the dense element matrices (for tests that assemble or inspect them). */
int or_force_elem_matrix(int p, int Q, const double *S_el, double *FE)
{
    or_basis bs;
    or_tab3 tb = {0};
    if (make_basis(p, Q, &bs)) return -1;
    if (make_tab3(&bs, &tb)) { free_tab3(&tb); return -3; }
    force_elem(&tb, S_el, 0, FE);
    free_tab3(&tb);
    return 0;
}

int or_mass_elem_matrix(int p, int Q, const double *mq_el, double *ME)
{
    or_basis bs;
    or_tab3 tb = {0};
    if (make_basis(p, Q, &bs)) return -1;
    if (make_tab3(&bs, &tb)) { free_tab3(&tb); return -3; }
    mass_elem(&tb, mq_el, 0, ME);
    free_tab3(&tb);
    return 0;
}

/* ------------------------------------------------------------ actions */

/*
 * y = F e (e == NULL means e = 1): y[c*N + g] = sum_E sum_i [R_E^T F_E e_E].
 * y is overwritten (zeroed first, then elements are added in ascending order).
 * With elems != NULL only the listed elements contribute.
 */
int or_force_mult(int n_elem, int p, int Q, int N, const int32_t *map, const double *S,
                  const double *e, const int32_t *elems, int n_sel, int absmode, double *y)
{
    or_basis bs;
    if (make_basis(p, Q, &bs)) return -1;
    const int D = bs.D, D3 = D * D * D, Dl3 = p * p * p, Q3 = Q * Q * Q;
    or_tab3 tb = {0};
    double *FE = (double *)malloc(sizeof(double) * 3 * D3 * Dl3);
    if (!FE || make_tab3(&bs, &tb)) { free(FE); free_tab3(&tb); return -3; }
    memset(y, 0, sizeof(double) * 3 * (size_t)N);
    for (int k = 0; k < NLOOP; ++k) {
        const int el = ELEM(k);
        force_elem(&tb, S + (size_t)el * 9 * Q3, absmode, FE);
        for (int c = 0; c < 3; ++c)
            for (int i = 0; i < D3; ++i) {
                double acc = 0.0;
                for (int j = 0; j < Dl3; ++j) {
                    double ej = e ? e[(size_t)el * Dl3 + j] : 1.0;
                    acc += FE[(c * D3 + i) * Dl3 + j] * (absmode ? fabs(ej) : ej);
                }
                y[(size_t)c * N + map[(size_t)el * D3 + i]] += acc;
            }
    }
    free(FE);
    free_tab3(&tb);
    return 0;
}

/* z = F^T v: z[E][j] = sum_{(i,c)} F_E[(i,c), j] v[c*N + g(i)]. Element-local, no scatter. */
int or_force_mult_T(int n_elem, int p, int Q, int N, const int32_t *map, const double *S,
                    const double *v, const int32_t *elems, int n_sel, int absmode, double *z)
{
    or_basis bs;
    if (make_basis(p, Q, &bs)) return -1;
    const int D = bs.D, D3 = D * D * D, Dl3 = p * p * p, Q3 = Q * Q * Q;
    or_tab3 tb = {0};
    double *FE = (double *)malloc(sizeof(double) * 3 * D3 * Dl3);
    if (!FE || make_tab3(&bs, &tb)) { free(FE); free_tab3(&tb); return -3; }
    for (int k = 0; k < NLOOP; ++k) {
        const int el = ELEM(k);
        force_elem(&tb, S + (size_t)el * 9 * Q3, absmode, FE);
        for (int j = 0; j < Dl3; ++j) {
            double acc = 0.0;
            for (int c = 0; c < 3; ++c)
                for (int i = 0; i < D3; ++i) {
                    double vi = v[(size_t)c * N + map[(size_t)el * D3 + i]];
                    acc += FE[(c * D3 + i) * Dl3 + j] * (absmode ? fabs(vi) : vi);
                }
            z[(size_t)el * Dl3 + j] = acc;
        }
    }
    free(FE);
    free_tab3(&tb);
    return 0;
}

/* y = M_v x, block diagonal over the 3 components: y_c = sum_E R^T M_E R x_c. */
int or_mass_mult(int n_elem, int p, int Q, int N, const int32_t *map, const double *mq,
                 const double *x, const int32_t *elems, int n_sel, int absmode, double *y)
{
    or_basis bs;
    if (make_basis(p, Q, &bs)) return -1;
    const int D = bs.D, D3 = D * D * D, Q3 = Q * Q * Q;
    or_tab3 tb = {0};
    double *ME = (double *)malloc(sizeof(double) * D3 * D3);
    if (!ME || make_tab3(&bs, &tb)) { free(ME); free_tab3(&tb); return -3; }
    memset(y, 0, sizeof(double) * 3 * (size_t)N);
    for (int k = 0; k < NLOOP; ++k) {
        const int el = ELEM(k);
        mass_elem(&tb, mq + (size_t)el * Q3, absmode, ME);
        for (int c = 0; c < 3; ++c)
            for (int i = 0; i < D3; ++i) {
                double acc = 0.0;
                for (int j = 0; j < D3; ++j) {
                    double xj = x[(size_t)c * N + map[(size_t)el * D3 + j]];
                    acc += ME[i * D3 + j] * (absmode ? fabs(xj) : xj);
                }
                y[(size_t)c * N + map[(size_t)el * D3 + i]] += acc;
            }
    }
    free(ME);
    free_tab3(&tb);
    return 0;
}

/* ------------------------------------------------- stiffness (diffusion) */

/*
 * Stiffness (diffusion) operator of the hyper-viscosity term (Sec. 2.1 names
 * the "stiffness matrix" operator the shock-capturing hyper-viscosity needs;
 * Sec. 6 the diffusion integrator used in the artificial-viscosity
 * calculations), on the kinematic H1 space, one block per velocity component
 * like M_v:
 *     K[i][j] = int kappa grad w_i . grad w_j dx
 *             = sum_q w_q kappa_q detJ_q (J_q^-T grad_xi w_i) . (J_q^-T grad_xi w_j)
 * on the current mesh x. kappa is given per quadrature point ([E][Q^3]) or
 * NULL for kappa = 1. The physical gradients are formed at each point
 * directly from the definition, the element matrix is dense, and
 * y_c = sum_E R_E^T K_E R_E u_c. With absmode the same loops run on
 * magnitudes (the scale of the rounding error).
 */
static void stiff_elem(const or_basis *bs, const or_tab3 *tb, const int32_t *nodes, int N,
                       const double *x, const double *kap_el, int absmode, double *KE)
{
    const int Q = bs->Q, D3 = tb->D3;
    memset(KE, 0, sizeof(double) * D3 * D3);
    double *gphys = (double *)malloc(sizeof(double) * 3 * D3);
    for (int qz = 0; qz < Q; ++qz)
    for (int qy = 0; qy < Q; ++qy)
    for (int qx = 0; qx < Q; ++qx) {
        const int q = qx + Q * (qy + Q * qz);
        const double w = bs->wq[qx] * bs->wq[qy] * bs->wq[qz];
        double J[3][3] = {{0}};
        for (int i = 0; i < D3; ++i) {
            const double *g = &tb->hg3[(q * D3 + i) * 3];
            for (int c = 0; c < 3; ++c)
                for (int d = 0; d < 3; ++d) J[c][d] += x[(size_t)c * N + nodes[i]] * g[d];
        }
        const double dJ = det3(J);
        double Ji[3][3];
        inv3(J, dJ, Ji);
        /* grad w_i = J^-T grad_xi w_i: component k = sum_d Ji[d][k] g[d] */
        for (int i = 0; i < D3; ++i) {
            const double *g = &tb->hg3[(q * D3 + i) * 3];
            for (int k = 0; k < 3; ++k)
                gphys[3 * i + k] = Ji[0][k] * g[0] + Ji[1][k] * g[1] + Ji[2][k] * g[2];
        }
        const double kap = kap_el ? kap_el[q] : 1.0;
        const double f = w * kap * dJ;
        for (int i = 0; i < D3; ++i)
            for (int j = 0; j < D3; ++j) {
                double s = 0.0;
                for (int k = 0; k < 3; ++k)
                    s += absmode ? fabs(gphys[3 * i + k]) * fabs(gphys[3 * j + k])
                                 : gphys[3 * i + k] * gphys[3 * j + k];
                KE[i * D3 + j] += absmode ? fabs(f) * s : f * s;
            }
    }
    free(gphys);
}

int or_stiff_elem_matrix(int p, int Q, int N, const int32_t *nodes, const double *x,
                         const double *kap_el, double *KE)
{
    or_basis bs;
    or_tab3 tb = {0};
    if (make_basis(p, Q, &bs)) return -1;
    if (make_tab3(&bs, &tb)) { free_tab3(&tb); return -3; }
    stiff_elem(&bs, &tb, nodes, N, x, kap_el, 0, KE);
    free_tab3(&tb);
    return 0;
}

/* y = K u for the three components of u ([3][N]); y overwritten. */
int or_stiff_mult(int n_elem, int p, int Q, int N, const int32_t *map, const double *x,
                  const double *kappa, const double *u, const int32_t *elems, int n_sel,
                  int absmode, double *y)
{
    or_basis bs;
    if (make_basis(p, Q, &bs)) return -1;
    const int D = bs.D, D3 = D * D * D, Q3 = Q * Q * Q;
    or_tab3 tb = {0};
    double *KE = (double *)malloc(sizeof(double) * D3 * D3);
    if (!KE || make_tab3(&bs, &tb)) { free(KE); free_tab3(&tb); return -3; }
    memset(y, 0, sizeof(double) * 3 * (size_t)N);
    for (int k = 0; k < NLOOP; ++k) {
        const int el = ELEM(k);
        const int32_t *nodes = map + (size_t)el * D3;
        stiff_elem(&bs, &tb, nodes, N, x, kappa ? kappa + (size_t)el * Q3 : NULL, absmode, KE);
        for (int c = 0; c < 3; ++c)
            for (int i = 0; i < D3; ++i) {
                double acc = 0.0;
                for (int j = 0; j < D3; ++j) {
                    const double uj = u[(size_t)c * N + nodes[j]];
                    acc += KE[i * D3 + j] * (absmode ? fabs(uj) : uj);
                }
                y[(size_t)c * N + nodes[i]] += acc;
            }
    }
    free(KE);
    free_tab3(&tb);
    return 0;
}

/* ------------------------------------------------------------- mass CG */

static double dot(const double *a, const double *b, size_t n)
{
    double s = 0.0;
    for (size_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/*
 * Unpreconditioned conjugate gradients (Hestenes-Stiefel) for M_v x = b with
 * x = 0 on the listed essential DOFs (indices into [3][N]); the other DOFs form
 * the free system. x holds the initial guess on entry (its essential entries
 * are zeroed). Stops when ||r|| <= rel_tol ||b_free||; reports the iteration
 * count and the true relative residual ||b_free - (M x)_free|| / ||b_free||.
 * Returns 0 when converged, 1 when max_iter was reached, <0 on errors.
 */
int or_mass_cg(int n_elem, int p, int Q, int N, const int32_t *map, const double *mq,
               const double *b, double *x, const int32_t *ess, int n_ess,
               double rel_tol, int max_iter, int *iters, double *rel_res)
{
    const size_t n = 3 * (size_t)N;
    double *r = (double *)malloc(sizeof(double) * n);
    double *d = (double *)malloc(sizeof(double) * n);
    double *Ad = (double *)malloc(sizeof(double) * n);
    unsigned char *fixed = (unsigned char *)calloc(n, 1);
    if (!r || !d || !Ad || !fixed) { free(r); free(d); free(Ad); free(fixed); return -3; }
    for (int k = 0; k < n_ess; ++k) fixed[ess[k]] = 1;
    for (size_t i = 0; i < n; ++i) if (fixed[i]) x[i] = 0.0;
    double bb = 0.0;
    for (size_t i = 0; i < n; ++i) if (!fixed[i]) bb += b[i] * b[i];
    or_mass_mult(n_elem, p, Q, N, map, mq, x, NULL, 0, 0, Ad);
    for (size_t i = 0; i < n; ++i) { r[i] = fixed[i] ? 0.0 : b[i] - Ad[i]; d[i] = r[i]; }
    double rr = dot(r, r, n);
    const double stop = rel_tol * rel_tol * bb;
    int it = 0, status = 1;
    if (rr <= stop) status = 0;
    while (status && it < max_iter) {
        or_mass_mult(n_elem, p, Q, N, map, mq, d, NULL, 0, 0, Ad);
        for (size_t i = 0; i < n; ++i) if (fixed[i]) Ad[i] = 0.0;
        const double alpha = rr / dot(d, Ad, n);
        for (size_t i = 0; i < n; ++i) { x[i] += alpha * d[i]; r[i] -= alpha * Ad[i]; }
        const double rr_new = dot(r, r, n);
        ++it;
        if (rr_new <= stop) { status = 0; rr = rr_new; break; }
        const double beta = rr_new / rr;
        rr = rr_new;
        for (size_t i = 0; i < n; ++i) d[i] = r[i] + beta * d[i];
    }
    or_mass_mult(n_elem, p, Q, N, map, mq, x, NULL, 0, 0, Ad);
    double res = 0.0;
    for (size_t i = 0; i < n; ++i)
        if (!fixed[i]) res += (b[i] - Ad[i]) * (b[i] - Ad[i]);
    *iters = it;
    *rel_res = bb > 0.0 ? sqrt(res / bb) : sqrt(res);
    free(r); free(d); free(Ad); free(fixed);
    return status;
}
