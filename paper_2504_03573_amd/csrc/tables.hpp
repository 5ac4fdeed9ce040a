// 1-D tables of the discretisation and their layout in one device array.
//
// All sum-factorised operators of the library are built from these 1-D
// matrices (Xia & Moxey, Sec. 3.1 basic operators; Sec. 3.2 trace
// evaluation):
//   B(P)    [n][N_P]  modes at the n = P+2 GLL points (BwdTrans rows, the
//                     transpose gives IProduct): Legendre P_i, or the modified
//                     C0 modes (Table 1 "Modal")
//   D(n)    [n][n]    collocation derivative l'_j(x_i) (PhysDeriv)
//   I(n,m)  [m][n]    Lagrange interpolation from n to m > n GLL points
//                     (gather + interpolate to the shared trace)
//   BF(m)   [m][PMAX+1], DBF(m): modes and their derivatives at m GLL points
//   X(n), W(n)        GLL nodes and weights
// A second set for Gauss (Gauss-Legendre) volume points has X, W, B and D at
// the n = P+2 Gauss points instead; I, BF and DBF (the shared trace stays on
// its GLL points) are the same in both sets.
#pragma once

namespace sipdg {

constexpr int PMAX = 8;          // highest supported order
constexpr int NMIN = 3;          // GLL points for p = 1
constexpr int NMAX = PMAX + 2;   // GLL points for p = PMAX
constexpr int NSLOT = NMAX * NMAX;

constexpr int tab_off_B(int P) {
    int o = 0;
    for (int q = 1; q < P; ++q) o += (q + 2) * (q + 1);
    return o;
}
constexpr int TAB_B_END = tab_off_B(PMAX + 1);
constexpr int tab_off_D(int n) {
    int o = TAB_B_END;
    for (int m = NMIN; m < n; ++m) o += m * m;
    return o;
}
constexpr int TAB_D_END = tab_off_D(NMAX + 1);
constexpr int NPAIR = NMAX - NMIN + 1;
constexpr int tab_off_I(int n, int m) { return TAB_D_END + ((n - NMIN) * NPAIR + (m - NMIN)) * NSLOT; }
constexpr int TAB_I_END = TAB_D_END + NPAIR * NPAIR * NSLOT;
constexpr int BF_SLOT = NMAX * (PMAX + 1);
constexpr int tab_off_BF(int m) { return TAB_I_END + (m - NMIN) * BF_SLOT; }
constexpr int TAB_BF_END = TAB_I_END + NPAIR * BF_SLOT;
constexpr int tab_off_DBF(int m) { return TAB_BF_END + (m - NMIN) * BF_SLOT; }
constexpr int TAB_DBF_END = TAB_BF_END + NPAIR * BF_SLOT;
constexpr int tab_off_X(int n) { return TAB_DBF_END + (n - NMIN) * NMAX; }
constexpr int tab_off_W(int n) { return TAB_DBF_END + NPAIR * NMAX + (n - NMIN) * NMAX; }
constexpr int TAB_SIZE = TAB_DBF_END + 2 * NPAIR * NMAX;

// Host: fill a TAB_SIZE array (FP64) for the given modal basis (0 Legendre,
// 1 modified C0; B, BF and DBF depend on it, the rest does not) and volume
// point set (gauss: Gauss-Legendre instead of GLL for X, W, B and D).
void build_tables(double *tab, int basis = 0, bool gauss = false);

// Host helpers also used by the topology/validation code.
void gll_nodes_weights(int n, double *x, double *w);
void gauss_nodes_weights(int n, double *x, double *w);

}  // namespace sipdg
