// Host construction of the 1-D tables (FP64).
//
// GLL nodes: the endpoints and the roots of P'_{n-1}, found by Newton's
// method from the Chebyshev-Gauss-Lobatto points; weights
// 2 / (n (n-1) P_{n-1}(x)^2).  Gauss nodes: the roots of P_n by Newton's
// method from the Chebyshev-Gauss points; weights 2 / ((1 - x^2) P'_n(x)^2).  Collocation derivative and interpolation use
// the barycentric form of Lagrange interpolation (Berrut & Trefethen 2004).
#include "tables.hpp"

#include <cmath>
#include <cstring>

namespace sipdg {

static void legendre_with_derivs(int p, double x, double *P, double *dP) {
    P[0] = 1.0;
    dP[0] = 0.0;
    if (p >= 1) {
        P[1] = x;
        dP[1] = 1.0;
    }
    for (int i = 1; i < p; ++i) {
        P[i + 1] = ((2 * i + 1) * x * P[i] - i * P[i - 1]) / (i + 1);
        dP[i + 1] = (i + 1) * P[i] + x * dP[i];
    }
}

void gll_nodes_weights(int n, double *x, double *w) {
    const int N = n - 1;  // polynomial degree of P_N
    double P[NMAX + 2], dP[NMAX + 2];
    x[0] = -1.0;
    x[N] = 1.0;
    for (int j = 1; j < N; ++j) {
        double t = -std::cos(M_PI * j / N);
        for (int it = 0; it < 100; ++it) {
            legendre_with_derivs(N, t, P, dP);
            // f = P'_N, f' = P''_N = (2 t P'_N - N (N+1) P_N) / (1 - t^2)
            double f = dP[N];
            double fp = (2.0 * t * dP[N] - N * (N + 1.0) * P[N]) / (1.0 - t * t);
            double dt = f / fp;
            t -= dt;
            if (std::fabs(dt) < 1e-17) break;
        }
        x[j] = t;
    }
    for (int j = 0; j < n / 2; ++j) {  // exact symmetry
        double s = 0.5 * (x[n - 1 - j] - x[j]);
        x[j] = -s;
        x[n - 1 - j] = s;
    }
    if (n % 2) x[n / 2] = 0.0;
    for (int j = 0; j < n; ++j) {
        legendre_with_derivs(N, x[j], P, dP);
        w[j] = 2.0 / (N * (N + 1.0) * P[N] * P[N]);
    }
}

void gauss_nodes_weights(int n, double *x, double *w) {
    double P[NMAX + 2], dP[NMAX + 2];
    for (int j = 0; j < n; ++j) {
        double t = -std::cos(M_PI * (j + 0.5) / n);
        for (int it = 0; it < 100; ++it) {
            legendre_with_derivs(n, t, P, dP);
            const double dt = P[n] / dP[n];
            t -= dt;
            if (std::fabs(dt) < 1e-17) break;
        }
        x[j] = t;
    }
    for (int j = 0; j < n / 2; ++j) {  // exact symmetry
        const double s = 0.5 * (x[n - 1 - j] - x[j]);
        x[j] = -s;
        x[n - 1 - j] = s;
    }
    if (n % 2) x[n / 2] = 0.0;
    for (int j = 0; j < n; ++j) {
        legendre_with_derivs(n, x[j], P, dP);
        w[j] = 2.0 / ((1.0 - x[j] * x[j]) * dP[n] * dP[n]);
    }
}

static void bary_weights(int n, const double *x, double *lam) {
    for (int j = 0; j < n; ++j) {
        double p = 1.0;
        for (int k = 0; k < n; ++k)
            if (k != j) p *= (x[j] - x[k]);
        lam[j] = 1.0 / p;
    }
}

// Modified C0 modal modes (Table 1 "Modal"; Karniadakis & Sherwin), vertex
// modes first: psi_0 = (1-x)/2, psi_1 = (1+x)/2, and for i >= 2 the bubble
// (1-x)/2 (1+x)/2 P^(1,1)_{i-2}(x).  With P^(1,1)_{i-2} = 2 P'_{i-1} / i and
// (1-x^2) P'_k = k(k+1)/(2k+1) (P_{k-1} - P_{k+1}) the bubble is
// (i-1) / (2(2i-1)) (P_{i-2} - P_i): here from the Legendre values P, dP
// (i <= p) into M, dM.
static void legendre_to_modal(int p, const double *P, const double *dP, double *M, double *dM) {
    M[0] = 0.5 * (P[0] - P[1]);
    dM[0] = 0.5 * (dP[0] - dP[1]);
    M[1] = 0.5 * (P[0] + P[1]);
    dM[1] = 0.5 * (dP[0] + dP[1]);
    for (int i = 2; i <= p; ++i) {
        const double c = (i - 1.0) / (2.0 * (2.0 * i - 1.0));
        M[i] = c * (P[i - 2] - P[i]);
        dM[i] = c * (dP[i - 2] - dP[i]);
    }
}

void build_tables(double *tab, int basis, bool gauss) {
    std::memset(tab, 0, sizeof(double) * TAB_SIZE);
    // X: the volume points (GLL or Gauss); G: the GLL points of the traces
    double X[NMAX + 1][NMAX], W[NMAX + 1][NMAX], G[NMAX + 1][NMAX], GW[NMAX + 1][NMAX];
    for (int n = NMIN; n <= NMAX; ++n) {
        gll_nodes_weights(n, G[n], GW[n]);
        if (gauss) gauss_nodes_weights(n, X[n], W[n]);
        else gll_nodes_weights(n, X[n], W[n]);
        for (int j = 0; j < n; ++j) {
            tab[tab_off_X(n) + j] = X[n][j];
            tab[tab_off_W(n) + j] = W[n][j];
        }
    }
    double P[PMAX + 2], dP[PMAX + 2];
    for (int Pd = 1; Pd <= PMAX; ++Pd) {
        int n = Pd + 2, np = Pd + 1;
        for (int q = 0; q < n; ++q) {
            legendre_with_derivs(Pd, X[n][q], P, dP);
            if (basis == 1) {
                double M[PMAX + 2], dM[PMAX + 2];
                legendre_to_modal(Pd, P, dP, M, dM);
                for (int i = 0; i < np; ++i) tab[tab_off_B(Pd) + q * np + i] = M[i];
                continue;
            }
            for (int i = 0; i < np; ++i) tab[tab_off_B(Pd) + q * np + i] = P[i];
        }
    }
    for (int n = NMIN; n <= NMAX; ++n) {
        double lam[NMAX];
        bary_weights(n, X[n], lam);
        double *D = tab + tab_off_D(n);
        for (int i = 0; i < n; ++i) {
            double diag = 0.0;
            for (int j = 0; j < n; ++j) {
                if (j == i) continue;
                double v = (lam[j] / lam[i]) / (X[n][i] - X[n][j]);
                D[i * n + j] = v;
                diag -= v;
            }
            D[i * n + i] = diag;
        }
        // interpolation between GLL sets (the fold of the GLL volume points
        // onto a finer trace; unused with Gauss volume points)
        double lg[NMAX];
        bary_weights(n, G[n], lg);
        for (int m = NMIN; m <= NMAX; ++m) {
            double *I = tab + tab_off_I(n, m);
            for (int t = 0; t < m; ++t) {
                double y = G[m][t];
                int hit = -1;
                for (int j = 0; j < n; ++j)
                    if (y == G[n][j]) hit = j;
                if (hit >= 0) {
                    for (int j = 0; j < n; ++j) I[t * n + j] = (j == hit) ? 1.0 : 0.0;
                    continue;
                }
                double den = 0.0;
                for (int j = 0; j < n; ++j) den += lg[j] / (y - G[n][j]);
                for (int j = 0; j < n; ++j) I[t * n + j] = (lg[j] / (y - G[n][j])) / den;
            }
        }
    }
    for (int m = NMIN; m <= NMAX; ++m) {
        for (int t = 0; t < m; ++t) {
            legendre_with_derivs(PMAX, G[m][t], P, dP);
            if (basis == 1) {
                double M[PMAX + 2], dM[PMAX + 2];
                legendre_to_modal(PMAX, P, dP, M, dM);
                for (int i = 0; i <= PMAX; ++i) {
                    P[i] = M[i];
                    dP[i] = dM[i];
                }
            }
            for (int i = 0; i <= PMAX; ++i) {
                tab[tab_off_BF(m) + t * (PMAX + 1) + i] = P[i];
                tab[tab_off_DBF(m) + t * (PMAX + 1) + i] = dP[i];
            }
        }
    }
}

}  // namespace sipdg
