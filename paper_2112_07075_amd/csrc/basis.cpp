// 1-D basis tables of the library (host side, FP64).
//
//   Gauss-Legendre points/weights on [0,1] (Sec. 3.4: standard Gauss-Legendre
//   quadrature): Newton on P_n; weight 2(1-s^2)/(n P_{n-1}(s))^2 on [-1,1].
//   Gauss-Lobatto points: roots of P_{p-1} - P_{p+1}, which vanishes exactly at
//   +-1 and the zeros of P_p' because (1-s^2) P_p' = p(p+1)/(2p+1) (P_{p-1} - P_{p+1});
//   its derivative is -(2p+1) P_p.
//   Lagrange values and derivatives: barycentric formulas (Berrut & Trefethen,
//   SIAM Review 2004), with the differentiation-matrix row when the evaluation
//   point is a node.
#include "basis.hpp"

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "kern_common.hpp"

namespace fepa {

// P_0..P_n at s
static void legendre_all(int n, double s, double *P)
{
    P[0] = 1.0;
    if (n >= 1) P[1] = s;
    for (int k = 1; k < n; ++k) P[k + 1] = ((2 * k + 1) * s * P[k] - k * P[k - 1]) / (k + 1);
}

void gauss_legendre01(int n, double *t, double *w)
{
    std::vector<double> P(n + 2);
    for (int k = 0; k < n; ++k) {
        // Tricomi-type first guess, descending order on [-1,1]
        double s = std::cos(M_PI * (4.0 * k + 3.0) / (4.0 * n + 2.0));
        for (int it = 0; it < 60; ++it) {
            legendre_all(n, s, P.data());
            const double dP = n * (P[n - 1] - s * P[n]) / (1.0 - s * s);
            const double step = P[n] / dP;
            s -= step;
            if (std::fabs(step) <= 1e-16 * std::fabs(s) + 1e-300) break;
        }
        legendre_all(n, s, P.data());
        const double wk = 2.0 * (1.0 - s * s) / ((n * P[n - 1]) * (n * P[n - 1]));
        // store ascending on [0,1]
        t[n - 1 - k] = 0.5 * (1.0 + s);
        w[n - 1 - k] = 0.5 * wk;
    }
}

void gauss_lobatto01(int p, double *t)
{
    std::vector<double> P(p + 2);
    t[0] = 0.0;
    t[p] = 1.0;
    for (int k = 1; k < p; ++k) {
        double s = -std::cos(M_PI * k / p);
        for (int it = 0; it < 60; ++it) {
            legendre_all(p + 1, s, P.data());
            const double f = P[p - 1] - P[p + 1];
            const double df = -(2.0 * p + 1.0) * P[p];
            const double step = f / df;
            s -= step;
            if (std::fabs(step) <= 1e-16) break;
        }
        t[k] = 0.5 * (1.0 + s);
    }
}

// values l_a(x) and derivatives l_a'(x) of the Lagrange basis on nodes t[0..n-1]
static void lagrange_bary(int n, const double *t, double x, double *val, double *der)
{
    std::vector<double> lam(n);
    for (int a = 0; a < n; ++a) {
        double d = 1.0;
        for (int b = 0; b < n; ++b)
            if (b != a) d *= (t[a] - t[b]);
        lam[a] = 1.0 / d;
    }
    int hit = -1;
    for (int a = 0; a < n; ++a)
        if (x == t[a]) hit = a;
    if (hit >= 0) {
        // differentiation-matrix row: D_ka = (lam_a/lam_k)/(t_k - t_a), D_kk = -sum of the rest
        double diag = 0.0;
        for (int a = 0; a < n; ++a) {
            val[a] = (a == hit) ? 1.0 : 0.0;
            if (a != hit) {
                der[a] = (lam[a] / lam[hit]) / (t[hit] - t[a]);
                diag -= der[a];
            }
        }
        der[hit] = diag;
        return;
    }
    double ell = 1.0;  // node polynomial prod (x - t_b)
    for (int b = 0; b < n; ++b) ell *= (x - t[b]);
    for (int a = 0; a < n; ++a) {
        val[a] = ell * lam[a] / (x - t[a]);
        double s = 0.0;
        for (int b = 0; b < n; ++b)
            if (b != a) s += 1.0 / (x - t[b]);
        der[a] = val[a] * s;
    }
}

std::vector<double> build_table(int p, int Q)
{
    const int D = p + 1, DL = p;
    std::vector<double> tq(Q), wq(Q), th(D), tl(DL), wl(DL), v(D), d(D), vl(DL), dl(DL);
    gauss_legendre01(Q, tq.data(), wq.data());
    gauss_lobatto01(p, th.data());
    gauss_legendre01(DL, tl.data(), wl.data());
    // layout: B[Q][D] | G[Q][D] | Bl[Q][DL] | W[Q]
    std::vector<double> tab(2 * Q * D + Q * DL + Q);
    for (int q = 0; q < Q; ++q) {
        lagrange_bary(D, th.data(), tq[q], v.data(), d.data());
        for (int i = 0; i < D; ++i) {
            tab[q * D + i] = v[i];
            tab[Q * D + q * D + i] = d[i];
        }
        lagrange_bary(DL, tl.data(), tq[q], vl.data(), dl.data());
        for (int j = 0; j < DL; ++j) tab[2 * Q * D + q * DL + j] = vl[j];
        tab[2 * Q * D + Q * DL + q] = wq[q];
    }
    return tab;
}

static uint16_t bf16_bits(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // NaN stays NaN
    u += 0x7fffu + ((u >> 16) & 1u);                                           // round to nearest even
    return (uint16_t)(u >> 16);
}

std::vector<unsigned char> build_mfma_table(int p, int Q, const std::vector<double> &tab)
{
    const int D = p + 1, DL = p;
    const MfmaLayout M = mfma_layout(D, Q);
    std::vector<unsigned char> out((size_t)M.bytes, 0);
    float *ft = (float *)out.data();
    for (size_t k = 0; k < tab.size() && (int)k < M.tabf; ++k) ft[k] = (float)tab[k];
    (void)DL;
    uint16_t *fr = (uint16_t *)(out.data() + (size_t)M.tabf * 4);
    const double *B = tab.data(), *G = tab.data() + Q * D;
    for (int ct = 0; ct < M.nt; ++ct)
        for (int d = 0; d < 3; ++d)
            for (int s = 0; s < M.ns; ++s)
                for (int l = 0; l < 64; ++l)
                    for (int j = 0; j < 8; ++j) {
                        const int q = s * 32 + (l / 16) * 8 + j, i = ct * 16 + l % 16;
                        double v = 0.0;
                        if (q < M.q3 && i < M.d3) {
                            const int qx = q % Q, qy = (q / Q) % Q, qz = q / (Q * Q);
                            const int ix = i % D, iy = (i / D) % D, iz = i / (D * D);
                            const double bx = B[qx * D + ix], by = B[qy * D + iy], bz = B[qz * D + iz];
                            const double gx = G[qx * D + ix], gy = G[qy * D + iy], gz = G[qz * D + iz];
                            v = d == 0 ? gx * by * bz : (d == 1 ? bx * gy * bz : bx * by * gz);
                        }
                        fr[((((size_t)ct * 3 + d) * M.ns + s) * 64 + l) * 8 + j] = bf16_bits((float)v);
                    }
    return out;
}

}  // namespace fepa
