// Host construction, in double precision, of the linear operators that
// complete the adjoint populations on the boundary ring (Sec. 2.5 and
// Appendix A of the paper).
//
// On a ring node with outward normal n the ALKS pull leaves the three
// populations with c_i.n > 0 undetermined. The paper fixes them, together
// with the Lagrange multipliers of the boundary conditions, as the
// least-squares (generalized-inverse) solution of the nine boundary
// equations, one per direction i:
//   flow     (n.c_i) f~_i - 2A sum_j w_j (n.c_j)(c_j.c_i) f~_j
//            + [mu~.c_i | lambda~ + mu~_s (c_i.t)] - kappa~ T (c_i.n) + s_i
//   thermal  (n.c_i) g~_i - B (n.q~) + [eta~ | kappa~ (c_i - u).n]
// (eq:afboundaryu, eq:afboundaryp, eq:afboundaryuq, eq:afboundarypq,
// eq:agboundaryT, eq:agboundaryq; the s~ and q~ of the printed conditions are
// expanded through eq:afs and eq:agq, and the reading of the garbled matrix
// M is the one that reproduces the printed closed form eq:ftilde).
// Everything except the zero-flux rows is independent of the node, so the
// solution is a fixed linear map of the known populations, the seed s and
// kappa~ T; the zero-flux case depends on the normal velocity u_n only
// through one column and is kept in Schur-complement form.
#include <cmath>
#include <cstring>

#include "lks_device.h"

namespace lks {
namespace {

const int HX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
const int HY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
const double HW[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                      1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

// D3Q19 in the numbering of the three-dimensional kernels
const int C19[19][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
                        {0, 0, 1},  {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                        {-1, 1, 0}, {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                        {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
const double W19[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                        1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                        1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

// inverse of an n x n matrix (n <= 8) by Gauss-Jordan with partial pivoting
void invert(int n, const double* a, double* inv) {
  double m[8][16];
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < 2 * n; ++c) m[r][c] = c < n ? a[r * n + c] : (c - n == r ? 1.0 : 0.0);
  for (int p = 0; p < n; ++p) {
    int piv = p;
    for (int r = p + 1; r < n; ++r)
      if (std::fabs(m[r][p]) > std::fabs(m[piv][p])) piv = r;
    if (piv != p)
      for (int c = 0; c < 2 * n; ++c) std::swap(m[p][c], m[piv][c]);
    const double d = m[p][p];
    for (int c = 0; c < 2 * n; ++c) m[p][c] /= d;
    for (int r = 0; r < n; ++r) {
      if (r == p) continue;
      const double f = m[r][p];
      for (int c = 0; c < 2 * n; ++c) m[r][c] -= f * m[p][c];
    }
  }
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) inv[r * n + c] = m[r][n + c];
}

// P = (K^T K)^-1 K^T for a rows x n matrix K (row-major), P is n x rows
void pseudo_inverse(int rows, int n, const double* K, double* P) {
  double G[64], Gi[64];
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      double s = 0;
      for (int r = 0; r < rows; ++r) s += K[r * n + a] * K[r * n + b];
      G[a * n + b] = s;
    }
  invert(n, G, Gi);
  for (int a = 0; a < n; ++a)
    for (int r = 0; r < rows; ++r) {
      double s = 0;
      for (int b = 0; b < n; ++b) s += Gi[a * n + b] * K[r * n + b];
      P[a * rows + r] = s;
    }
}

}  // namespace

void build_ring_ops(double A, double Bf, RingOp ops[4]) {
  const int NRM[4][2] = {{-1, 0}, {1, 0}, {0, -1}, {0, 1}};
  for (int o = 0; o < 4; ++o) {
    RingOp& op = ops[o];
    std::memset(&op, 0, sizeof op);
    const int nx = NRM[o][0], ny = NRM[o][1];
    const int tx = -ny, ty = nx;
    int cn[9], nu = 0;
    for (int q = 0; q < 9; ++q) {
      cn[q] = HX[q] * nx + HY[q] * ny;
      if (cn[q] > 0) op.unk[nu++] = q;
    }
    for (int a = 0; a < 3; ++a) {
      op.uw[a] = HW[op.unk[a]];
      op.ucx[a] = HX[op.unk[a]];
      op.ucy[a] = HY[op.unk[a]];
    }
    // flow rows: coefficient of f~_q in row r
    double M[9][9];
    for (int r = 0; r < 9; ++r)
      for (int q = 0; q < 9; ++q)
        M[r][q] = (r == q ? cn[r] : 0.0) -
                  2.0 * A * HW[q] * cn[q] * double(HX[q] * HX[r] + HY[q] * HY[r]);
    for (int v = 0; v < 2; ++v) {
      double K[9 * 5], P[5 * 9];
      for (int r = 0; r < 9; ++r) {
        for (int a = 0; a < 3; ++a) K[r * 5 + a] = M[r][op.unk[a]];
        K[r * 5 + 3] = v == 0 ? double(HX[r]) : 1.0;
        K[r * 5 + 4] = v == 0 ? double(HY[r]) : double(HX[r] * tx + HY[r] * ty);
      }
      pseudo_inverse(9, 5, K, P);
      for (int a = 0; a < 3; ++a) {
        double s = 0, k = 0;
        for (int r = 0; r < 9; ++r) {
          s += P[a * 9 + r];
          k += P[a * 9 + r] * cn[r];
        }
        op.Ls[v][a] = -s;
        op.Lk[v][a] = k;
        for (int q = 0; q < 9; ++q) {
          double t = 0;
          if (cn[q] <= 0)
            for (int r = 0; r < 9; ++r) t += P[a * 9 + r] * M[r][q];
          op.Lf[v][a][q] = -t;
        }
      }
    }
    // thermal rows: coefficient of g~_q in row r
    double Mg[9][9];
    for (int r = 0; r < 9; ++r)
      for (int q = 0; q < 9; ++q) Mg[r][q] = (r == q ? cn[r] : 0.0) - Bf * HW[q] * cn[q];
    {
      double K[9 * 4], P[4 * 9];
      for (int r = 0; r < 9; ++r) {
        for (int a = 0; a < 3; ++a) K[r * 4 + a] = Mg[r][op.unk[a]];
        K[r * 4 + 3] = 1.0;
      }
      pseudo_inverse(9, 4, K, P);
      for (int a = 0; a < 3; ++a)
        for (int q = 0; q < 9; ++q) {
          double t = 0;
          if (cn[q] <= 0)
            for (int r = 0; r < 9; ++r) t += P[a * 9 + r] * Mg[r][q];
          op.Ld[a][q] = -t;
        }
    }
    {
      double K0[9 * 3], G[9], H[9];
      for (int r = 0; r < 9; ++r)
        for (int a = 0; a < 3; ++a) K0[r * 3 + a] = Mg[r][op.unk[a]];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          double s = 0;
          for (int r = 0; r < 9; ++r) s += K0[r * 3 + a] * K0[r * 3 + b];
          G[a * 3 + b] = s;
        }
      invert(3, G, H);
      // HK = H K0^T (3 x 9); Q = I - K0 HK (9 x 9)
      double HK[3 * 9], Q[9][9];
      for (int a = 0; a < 3; ++a)
        for (int r = 0; r < 9; ++r) {
          double s = 0;
          for (int b = 0; b < 3; ++b) s += H[a * 3 + b] * K0[r * 3 + b];
          HK[a * 9 + r] = s;
        }
      for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 9; ++c) {
          double s = 0;
          for (int a = 0; a < 3; ++a) s += K0[r * 3 + a] * HK[a * 9 + c];
          Q[r][c] = (r == c ? 1.0 : 0.0) - s;
        }
      double Qcn[9], Q1[9];
      for (int r = 0; r < 9; ++r) {
        double s = 0, t = 0;
        for (int c = 0; c < 9; ++c) {
          s += Q[r][c] * cn[c];
          t += Q[r][c];
        }
        Qcn[r] = s;
        Q1[r] = t;
      }
      op.A0 = op.A1 = op.A2 = 0;
      for (int r = 0; r < 9; ++r) {
        op.A0 += cn[r] * Qcn[r];
        op.A1 += cn[r] * Q1[r];
        op.A2 += Q1[r];
      }
      for (int q = 0; q < 9; ++q) {
        double ga = 0, ge = 0;
        if (cn[q] <= 0)
          for (int r = 0; r < 9; ++r) {
            ga += Qcn[r] * Mg[r][q];
            ge += Q1[r] * Mg[r][q];
          }
        op.ga[q] = ga;
        op.ge[q] = ge;
      }
      for (int a = 0; a < 3; ++a) {
        double hc = 0, h1 = 0;
        for (int r = 0; r < 9; ++r) {
          hc += HK[a * 9 + r] * cn[r];
          h1 += HK[a * 9 + r];
        }
        op.hc[a] = hc;
        op.h1[a] = h1;
        for (int q = 0; q < 9; ++q) {
          double t = 0;
          if (cn[q] <= 0)
            for (int r = 0; r < 9; ++r) t += HK[a * 9 + r] * Mg[r][q];
          op.Lg0[a][q] = -t;
        }
      }
    }
  }
}

// D3Q19 faces: the same least-squares completion over 19 rows, with the five
// directions c_i.n > 0 unknown; the pressure face has the multipliers
// lambda~ + mu~_1 (c_i.t1) + mu~_2 (c_i.t2) with t1, t2 the two coordinate
// axes normal to n, the velocity face mu~.c_i.
void build_face_ops3(double A, double Bf, FaceOp3 ops[6]) {
  for (int o = 0; o < 6; ++o) {
    FaceOp3& op = ops[o];
    std::memset(&op, 0, sizeof op);
    const int ax = o / 2, sg = (o & 1) ? 1 : -1;
    const int t1 = (ax + 1) % 3, t2 = (ax + 2) % 3;
    int cn[19], nu = 0;
    for (int q = 0; q < 19; ++q) {
      cn[q] = sg * C19[q][ax];
      if (cn[q] > 0) op.unk[nu++] = q;
    }
    for (int a = 0; a < 5; ++a) {
      op.uw[a] = W19[op.unk[a]];
      for (int d = 0; d < 3; ++d) op.uc[a][d] = C19[op.unk[a]][d];
    }
    double M[19][19];
    for (int r = 0; r < 19; ++r)
      for (int q = 0; q < 19; ++q) {
        const double cc = C19[q][0] * C19[r][0] + C19[q][1] * C19[r][1] + C19[q][2] * C19[r][2];
        M[r][q] = (r == q ? cn[r] : 0.0) - 2.0 * A * W19[q] * cn[q] * cc;
      }
    for (int v = 0; v < 2; ++v) {
      double K[19 * 8], P[8 * 19];
      for (int r = 0; r < 19; ++r) {
        for (int a = 0; a < 5; ++a) K[r * 8 + a] = M[r][op.unk[a]];
        if (v == 0) {
          for (int d = 0; d < 3; ++d) K[r * 8 + 5 + d] = C19[r][d];
        } else {
          K[r * 8 + 5] = 1.0;
          K[r * 8 + 6] = C19[r][t1];
          K[r * 8 + 7] = C19[r][t2];
        }
      }
      pseudo_inverse(19, 8, K, P);
      for (int a = 0; a < 5; ++a) {
        double s = 0, k = 0;
        for (int r = 0; r < 19; ++r) {
          s += P[a * 19 + r];
          k += P[a * 19 + r] * cn[r];
        }
        op.Ls[v][a] = -s;
        op.Lk[v][a] = k;
        for (int q = 0; q < 19; ++q) {
          double t = 0;
          if (cn[q] <= 0)
            for (int r = 0; r < 19; ++r) t += P[a * 19 + r] * M[r][q];
          op.Lf[v][a][q] = -t;
        }
      }
    }
    double Mg[19][19];
    for (int r = 0; r < 19; ++r)
      for (int q = 0; q < 19; ++q) Mg[r][q] = (r == q ? cn[r] : 0.0) - Bf * W19[q] * cn[q];
    {
      double K[19 * 6], P[6 * 19];
      for (int r = 0; r < 19; ++r) {
        for (int a = 0; a < 5; ++a) K[r * 6 + a] = Mg[r][op.unk[a]];
        K[r * 6 + 5] = 1.0;
      }
      pseudo_inverse(19, 6, K, P);
      for (int a = 0; a < 5; ++a)
        for (int q = 0; q < 19; ++q) {
          double t = 0;
          if (cn[q] <= 0)
            for (int r = 0; r < 19; ++r) t += P[a * 19 + r] * Mg[r][q];
          op.Ld[a][q] = -t;
        }
    }
    {
      // zero-flux face: Schur form in the normal velocity u_n
      double K0[19 * 5], G[25], H[25], HK[5 * 19];
      for (int r = 0; r < 19; ++r)
        for (int a = 0; a < 5; ++a) K0[r * 5 + a] = Mg[r][op.unk[a]];
      for (int a = 0; a < 5; ++a)
        for (int b = 0; b < 5; ++b) {
          double s = 0;
          for (int r = 0; r < 19; ++r) s += K0[r * 5 + a] * K0[r * 5 + b];
          G[a * 5 + b] = s;
        }
      invert(5, G, H);
      for (int a = 0; a < 5; ++a)
        for (int r = 0; r < 19; ++r) {
          double s = 0;
          for (int b = 0; b < 5; ++b) s += H[a * 5 + b] * K0[r * 5 + b];
          HK[a * 19 + r] = s;
        }
      double Qcn[19], Q1[19];
      for (int r = 0; r < 19; ++r) {
        double s = 0, t = 0;
        for (int c = 0; c < 19; ++c) {
          double kk = 0;
          for (int a = 0; a < 5; ++a) kk += K0[r * 5 + a] * HK[a * 19 + c];
          const double q = (r == c ? 1.0 : 0.0) - kk;
          s += q * cn[c];
          t += q;
        }
        Qcn[r] = s;
        Q1[r] = t;
      }
      op.A0 = op.A1 = op.A2 = 0;
      for (int r = 0; r < 19; ++r) {
        op.A0 += cn[r] * Qcn[r];
        op.A1 += cn[r] * Q1[r];
        op.A2 += Q1[r];
      }
      for (int q = 0; q < 19; ++q) {
        double ga = 0, ge = 0;
        if (cn[q] <= 0)
          for (int r = 0; r < 19; ++r) {
            ga += Qcn[r] * Mg[r][q];
            ge += Q1[r] * Mg[r][q];
          }
        op.ga[q] = ga;
        op.ge[q] = ge;
      }
      for (int a = 0; a < 5; ++a) {
        double hc = 0, h1 = 0;
        for (int r = 0; r < 19; ++r) {
          hc += HK[a * 19 + r] * cn[r];
          h1 += HK[a * 19 + r];
        }
        op.hc[a] = hc;
        op.h1[a] = h1;
        for (int q = 0; q < 19; ++q) {
          double t = 0;
          if (cn[q] <= 0)
            for (int r = 0; r < 19; ++r) t += HK[a * 19 + r] * Mg[r][q];
          op.Lg0[a][q] = -t;
        }
      }
    }
  }
}

}  // namespace lks
