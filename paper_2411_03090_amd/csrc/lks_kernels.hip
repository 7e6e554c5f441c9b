// HIP kernels of the LKS forward step and the ALKS adjoint step on gfx950.
//
// Both steps are memory-bound gathers over a structure-of-arrays state
// (one contiguous array per field, x fastest). A workgroup of 256 threads
// owns a 64 x 4 tile:
//   stage A  every node of the tile plus a 1-node halo computes what its
//            neighbours will pull from it and stores it in LDS;
//   stage B  every tile node pulls from its 8 neighbours in LDS, applies the
//            local terms and writes its new state with coalesced stores.
// Nothing is a dense contraction, so there is no MFMA; reductions use
// wavefront shuffles and a fixed per-tile order, so every result is
// deterministic run to run (the checkpoint replay relies on it).
#include "lks_device.h"

namespace lks {

// D2Q9 velocities and weights (Sec. 2.3, eq:D2Q9w)
__device__ constexpr int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr double WD[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

__device__ inline int wrapi(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// Second-order central difference inside, second-order one-sided difference
// at the two ends of an axis (the boundary normal, and both axes at
// corners), wrap-around in a periodic box. `at(o)` returns the field at
// offset o along the axis.
template <typename R, typename F>
__device__ inline R fd_axis(int p, int n, int periodic, F at) {
  if (periodic || (p > 0 && p < n - 1)) return R(0.5) * (at(1) - at(-1));
  if (p == 0) return R(0.5) * (R(-3) * at(0) + R(4) * at(1) - at(2));
  return R(0.5) * (R(3) * at(0) - R(4) * at(-1) + at(-2));
}

template <typename R>
__device__ inline R gdx(const R* __restrict__ f, int i, int j, const Geo& g) {
  const int row = j * g.nx;
  return fd_axis<R>(i, g.nx, g.periodic,
                    [&](int o) { return f[row + wrapi(i + o, g.nx)]; });
}
template <typename R>
__device__ inline R gdy(const R* __restrict__ f, int i, int j, const Geo& g) {
  return fd_axis<R>(j, g.ny, g.periodic,
                    [&](int o) { return f[wrapi(j + o, g.ny) * g.nx + i]; });
}

// ---------------------------------------------------------------------------
// design -> coefficients (eq:brinkman, eq:conductivity, eq:B)
// ---------------------------------------------------------------------------
template <typename R>
__global__ void coef_kernel(Geo g, const double* __restrict__ gamma, double amax, double qa,
                            double Kf, double Ks, double qk, R* __restrict__ inv1pa,
                            R* __restrict__ B, R* __restrict__ dA3, R* __restrict__ dB) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.N) return;
  int i = k % g.nx, j = k / g.nx;
  bool ring = !g.periodic && (i == 0 || j == 0 || i == g.nx - 1 || j == g.ny - 1);
  if (ring) {
    inv1pa[k] = R(1);
    B[k] = R(g.Bf);
    dA3[k] = R(0);
    dB[k] = R(0);
    return;
  }
  double ga = gamma[k];
  double alpha = amax * qa * (1.0 - ga) / (qa + ga);
  double dalpha = -amax * qa * (1.0 + qa) / ((qa + ga) * (qa + ga));
  double K = Kf + (Ks - Kf) * qk * (1.0 - ga) / (qk + ga);
  double dK = -(Ks - Kf) * qk * (1.0 + qk) / ((qk + ga) * (qk + ga));
  inv1pa[k] = R(1.0 / (1.0 + alpha));
  B[k] = R(3.0 * (1.0 / 6.0 - K));
  dA3[k] = R(3.0 * dalpha);
  dB[k] = R(-3.0 * dK);
}

// ---------------------------------------------------------------------------
// level-0 state
// ---------------------------------------------------------------------------
template <typename R>
__global__ void init_kernel(Geo g, const uint8_t* __restrict__ mask, const R* __restrict__ ubx,
                            const R* __restrict__ uby, const R* __restrict__ Tb, double fac0,
                            R* __restrict__ d, R* __restrict__ ux, R* __restrict__ uy,
                            R* __restrict__ T) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.N) return;
  d[k] = R(0);
  R vx = R(0), vy = R(0), t = R(0);
  if (!g.periodic) {
    int m = mask[k];
    if ((m & 3) == FLOW_VELOCITY) {
      vx = R(double(ubx[k]) * fac0);
      vy = R(double(uby[k]) * fac0);
    }
    if (g.thermal) {
      int mt = m;
      int kt = k;
      if ((m & 3) == FLOW_CORNER) {  // corners take their y-neighbour's value
        int i = k % g.nx, j = k / g.nx;
        kt = (j == 0 ? 1 : g.ny - 2) * g.nx + i;
        mt = mask[kt];
      }
      if (((mt >> 2) & 3) == THERM_DIRICHLET) t = Tb[kt];
    }
  }
  ux[k] = vx;
  uy[k] = vy;
  if (g.thermal) T[k] = t;
}

// ---------------------------------------------------------------------------
// block reduction helper (deterministic)
// ---------------------------------------------------------------------------
__device__ inline double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < NTHREADS / 64; ++w) s += red[w];
  return s;
}

// ---------------------------------------------------------------------------
// LKS step
// ---------------------------------------------------------------------------
// One LKS step, level n -> n+1 (eq:rho, eq:u, eq:T with eq:feq2 and eq:geq2
// read as g_i^eq = w_i [T (1 + 3 c.u) + B c.grad T], and the implicit
// Brinkman term of eq:lbef_ex giving u = U* / (1 + alpha)).
// Density is carried as drho = rho - 1: the constant part of f_i^eq adds 1
// to the density and 0 to the momentum, so LDS holds f'_i = f_i^eq - w_i.
// Boundary nodes complete the density (velocity node), normal velocity
// (pressure node) or temperature (adiabatic node) from the moment balance of
// the pulled populations; corners copy density and temperature from their
// y-neighbour, whose thread writes them.
template <typename R, bool TH>
__global__ __launch_bounds__(NTHREADS) void lks_step_kernel(Geo g, FwdArgs<R> a) {
  __shared__ R sf[9][LPOS];
  __shared__ R sg[TH ? 9 : 1][TH ? LPOS : 1];
  __shared__ double red[NTHREADS / 64];

  int x0, x1, y0, y1;
  tile_extent(blockIdx.x, g.ntx, g.nx, TX, &x0, &x1);
  tile_extent(blockIdx.y, g.nty, g.ny, TY, &y0, &y1);
  const int tw = x1 - x0, th = y1 - y0, hw = tw + 2, hh = th + 2;
  const R A = R(g.A);

  // stage A: post-collision populations of the tile and its halo
  for (int p = threadIdx.x; p < hw * hh; p += NTHREADS) {
    int lx = p % hw, ly = p / hw;
    int i = x0 + lx - 1, j = y0 + ly - 1;
    if (g.periodic) {
      i = wrapi(i, g.nx);
      j = wrapi(j, g.ny);
    } else if (i < 0 || j < 0 || i >= g.nx || j >= g.ny) {
      continue;
    }
    const int k = j * g.nx + i;
    const int pos = ly * LW + lx;
    const R d = a.d0[k], ux = a.ux0[k], uy = a.uy0[k];
    const R uxx = gdx(a.ux0, i, j, g), uxy = gdy(a.ux0, i, j, g);
    const R uyx = gdx(a.uy0, i, j, g), uyy = gdy(a.uy0, i, j, g);
    // f'_i = w_i [P + 3 c.u + cx^2 Xx + cy^2 Yy + cx cy Xy]
    const R P = d - R(1.5) * (ux * ux + uy * uy);
    const R Xx = R(4.5) * ux * ux + R(2) * A * uxx;
    const R Yy = R(4.5) * uy * uy + R(2) * A * uyy;
    const R Xy = R(9) * ux * uy + R(2) * A * (uxy + uyx);
    const R u3x = R(3) * ux, u3y = R(3) * uy;
    const R w0 = R(4.0 / 9), w1 = R(1.0 / 9), w5 = R(1.0 / 36);
    const R diag = P + Xx + Yy;
    sf[0][pos] = w0 * P;
    sf[1][pos] = w1 * (P + u3x + Xx);
    sf[2][pos] = w1 * (P + u3y + Yy);
    sf[3][pos] = w1 * (P - u3x + Xx);
    sf[4][pos] = w1 * (P - u3y + Yy);
    sf[5][pos] = w5 * (diag + u3x + u3y + Xy);
    sf[6][pos] = w5 * (diag - u3x + u3y - Xy);
    sf[7][pos] = w5 * (diag - u3x - u3y + Xy);
    sf[8][pos] = w5 * (diag + u3x - u3y - Xy);
    if constexpr (TH) {
      const R T = a.T0[k];
      const R Bk = a.B[k];
      const R Wx = R(3) * T * ux + Bk * gdx(a.T0, i, j, g);
      const R Wy = R(3) * T * uy + Bk * gdy(a.T0, i, j, g);
      sg[0][pos] = w0 * T;
      sg[1][pos] = w1 * (T + Wx);
      sg[2][pos] = w1 * (T + Wy);
      sg[3][pos] = w1 * (T - Wx);
      sg[4][pos] = w1 * (T - Wy);
      sg[5][pos] = w5 * (T + Wx + Wy);
      sg[6][pos] = w5 * (T - Wx + Wy);
      sg[7][pos] = w5 * (T - Wx - Wy);
      sg[8][pos] = w5 * (T + Wx - Wy);
    }
  }
  __syncthreads();

  // stage B: pull and close
  double part = 0.0;
  for (int p = threadIdx.x; p < tw * th; p += NTHREADS) {
    const int lx = p % tw, ly = p / tw;
    const int i = x0 + lx, j = y0 + ly;
    const int k = j * g.nx + i;
    const int pos = (ly + 1) * LW + (lx + 1);
    const int m = a.mask[k];
    const int fc = g.periodic ? FLOW_INTERIOR : (m & 3);
    if (fc == FLOW_CORNER) continue;
    R f[9], gg[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) f[q] = sf[q][pos - CX[q] - CY[q] * LW];
    if constexpr (TH) {
#pragma unroll
      for (int q = 0; q < 9; ++q) gg[q] = sg[q][pos - CX[q] - CY[q] * LW];
    }
    R dn, uxn, uyn, Tn = R(0);
    if (fc == FLOW_INTERIOR) {
      dn = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
      const R Ux = f[1] - f[3] + f[5] - f[6] - f[7] + f[8];
      const R Uy = f[2] - f[4] + f[5] + f[6] - f[7] - f[8];
      const R s = a.inv1pa[k];
      uxn = Ux * s;
      uyn = Uy * s;
      if constexpr (TH) Tn = gg[0] + gg[1] + gg[2] + gg[3] + gg[4] + gg[5] + gg[6] + gg[7] + gg[8];
    } else {
      const int nx_ = (i == 0) ? -1 : (i == g.nx - 1 ? 1 : 0);
      const int ny_ = nx_ != 0 ? 0 : (j == 0 ? -1 : 1);
      R S0 = R(0), Sp = R(0), S0g = R(0), Spg = R(0);
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const int cn = CX[q] * nx_ + CY[q] * ny_;
        if (cn == 0) {
          S0 += f[q];
          if constexpr (TH) S0g += gg[q];
        } else if (cn > 0) {
          Sp += f[q];
          if constexpr (TH) Spg += gg[q];
        }
      }
      R un;
      if (fc == FLOW_VELOCITY) {
        const double fac = a.ufac[a.level_out];
        uxn = R(double(a.ubx[k]) * fac);
        uyn = R(double(a.uby[k]) * fac);
        un = uxn * R(nx_) + uyn * R(ny_);
        dn = S0 + R(2) * Sp - un;
      } else {
        const R dout = R(g.drho_out);
        dn = dout;
        un = S0 + R(2) * Sp - dout;
        uxn = un * R(nx_);
        uyn = un * R(ny_);
      }
      if constexpr (TH) {
        if (((m >> 2) & 3) == THERM_DIRICHLET) Tn = a.Tb[k];
        else Tn = (S0g + R(2) * Spg) / (R(1) + un);
      }
      // the y-neighbour of a corner writes the corner
      if (i == 0 || i == g.nx - 1) {
        if (j == 1) {
          const int kc = i;
          a.d1[kc] = dn;
          a.ux1[kc] = R(0);
          a.uy1[kc] = R(0);
          if constexpr (TH) a.T1[kc] = Tn;
        }
        if (j == g.ny - 2) {
          const int kc = (g.ny - 1) * g.nx + i;
          a.d1[kc] = dn;
          a.ux1[kc] = R(0);
          a.uy1[kc] = R(0);
          if constexpr (TH) a.T1[kc] = Tn;
        }
      }
    }
    a.d1[k] = dn;
    a.ux1[k] = uxn;
    a.uy1[k] = uyn;
    if constexpr (TH) a.T1[k] = Tn;
    if (a.acc) {
      if (a.objective == 1) {
        if (m & TAG_PROBE) part += double(uxn) * double(Tn);
      } else {
        if (m & TAG_J_INLET) part += double(dn);
        if (m & TAG_J_OUTLET) part -= double(dn);
      }
    }
  }
  if (a.acc) {
    double s = block_sum(part, red);
    if (threadIdx.x == 0) a.acc[blockIdx.y * g.ntx + blockIdx.x] += s;
  }
}

// ---------------------------------------------------------------------------
// adjoint boundary fill (double precision, per ring node)
// ---------------------------------------------------------------------------
// Solve min ||K x + b|| through the normal equations K^T K x = -K^T b with a
// Cholesky factorisation; C <= 5 unknowns.
template <int C>
struct Normal {
  double G[C][C];
  double h[C];
  __device__ void zero() {
#pragma unroll
    for (int r = 0; r < C; ++r) {
      h[r] = 0.0;
#pragma unroll
      for (int c = 0; c < C; ++c) G[r][c] = 0.0;
    }
  }
  __device__ void row(const double (&k)[C], double b) {
#pragma unroll
    for (int r = 0; r < C; ++r) {
      h[r] += k[r] * b;
#pragma unroll
      for (int c = 0; c <= r; ++c) G[r][c] += k[r] * k[c];
    }
  }
  __device__ void solve(double (&x)[C]) {
    double L[C][C];
#pragma unroll
    for (int r = 0; r < C; ++r) {
#pragma unroll
      for (int c = 0; c <= r; ++c) {
        double s = G[r][c];
#pragma unroll
        for (int t = 0; t < c; ++t) s -= L[r][t] * L[c][t];
        L[r][c] = (r == c) ? sqrt(s) : s / L[c][c];
      }
    }
    double y[C];
#pragma unroll
    for (int r = 0; r < C; ++r) {
      double s = -h[r];
#pragma unroll
      for (int t = 0; t < r; ++t) s -= L[r][t] * y[t];
      y[r] = s / L[r][r];
    }
#pragma unroll
    for (int r = C - 1; r >= 0; --r) {
      double s = y[r];
#pragma unroll
      for (int t = r + 1; t < C; ++t) s -= L[t][r] * x[t];
      x[r] = s / L[r][r];
    }
  }
};

// Least-squares completion of the adjoint populations at a ring node
// (Sec. 2.5, Appendix A). With outward normal n, the pulled values are known
// for c_i.n <= 0; the three with c_i.n > 0 and the multipliers minimise,
// over all nine rows i,
//   flow:    (n.c_i) f~_i - 2A sum_j w_j (n.c_j)(c_j.c_i) f~_j
//            + [mu~.c_i | lambda~ + mu~_s (c_i.t)] - kappa~ T (c_i.n) + s_i
//   thermal: (n.c_i) g~_i - B (n.q~) + [eta~ | kappa~ (c_i - u).n]
// (eq:afboundaryu, eq:afboundaryp, eq:agboundaryT, eq:afboundaryuq,
// eq:afboundarypq, eq:agboundaryq with s~ and q~ expanded through eq:afs and
// eq:agq). The thermal system is solved first; its kappa~ enters the flow
// rows of a flux node as a known term. s_i = dJ_dO/df_i: +seed/3 on inlet
// nodes and -seed/3 on outlet nodes of the pressure drop (p = sum f_i / 3).
// Returns the raw moments rho~, U~, s~ (xx, xy, yy), T~, q~ of the
// completed set.
template <typename R, bool TH>
__device__ void ring_fill(const Geo& g, const AdjArgs<R>& a, int i, int j, int k, int m,
                          double mom[9]) {
  const int nx_ = (i == 0) ? -1 : (i == g.nx - 1 ? 1 : 0);
  const int ny_ = nx_ != 0 ? 0 : (j == 0 ? -1 : 1);
  double f[9], gq[9];
  int cn[9];
  int uq[3], nu = 0;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    cn[q] = CX[q] * nx_ + CY[q] * ny_;
    f[q] = 0.0;
    gq[q] = 0.0;
    if (cn[q] <= 0) {
      const int kz = (j + CY[q]) * g.nx + (i + CX[q]);
      f[q] = double(a.r0[kz]) + CX[q] * double(a.vx0[kz]) + CY[q] * double(a.vy0[kz]);
      if constexpr (TH) gq[q] = double(a.th0[kz]);
    } else {
      uq[nu++] = q;
    }
  }
  double kappa = 0.0;
  const int tclass = (m >> 2) & 3;
  const bool flux = TH && tclass == THERM_FLUX;
  if constexpr (TH) {
    const double Bn = double(a.B[k]);
    const double un = double(a.ux[k]) * nx_ + double(a.uy[k]) * ny_;
    double Qk = 0.0;
#pragma unroll
    for (int q = 0; q < 9; ++q)
      if (cn[q] <= 0) Qk += WD[q] * cn[q] * gq[q];
    Normal<4> ne;
    ne.zero();
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      double kr[4];
#pragma unroll
      for (int c = 0; c < 3; ++c) kr[c] = (uq[c] == r ? double(cn[r]) : 0.0) - Bn * WD[uq[c]];
      kr[3] = flux ? double(cn[r]) - un : 1.0;
      const double b = (cn[r] <= 0 ? cn[r] * gq[r] : 0.0) - Bn * Qk;
      ne.row(kr, b);
    }
    double x[4];
    ne.solve(x);
#pragma unroll
    for (int c = 0; c < 3; ++c) gq[uq[c]] = x[c];
    if (flux) kappa = x[3];
  }
  {
    const double A = g.A;
    double Mx = 0.0, My = 0.0;
#pragma unroll
    for (int q = 0; q < 9; ++q)
      if (cn[q] <= 0) {
        Mx += WD[q] * cn[q] * CX[q] * f[q];
        My += WD[q] * cn[q] * CY[q] * f[q];
      }
    double s = 0.0;
    if (m & TAG_J_INLET) s += a.seed_dp / 3.0;
    if (m & TAG_J_OUTLET) s -= a.seed_dp / 3.0;
    const double Tn = TH ? double(a.T[k]) : 0.0;
    const bool vel = (m & 3) == FLOW_VELOCITY;
    const int tx_ = -ny_, ty_ = nx_;
    Normal<5> ne;
    ne.zero();
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      double kr[5];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int q = uq[c];
        kr[c] = (q == r ? double(cn[r]) : 0.0) -
                2.0 * A * WD[q] * double(CX[q] * CX[r] + CY[q] * CY[r]);
      }
      kr[3] = vel ? double(CX[r]) : 1.0;
      kr[4] = vel ? double(CY[r]) : double(CX[r] * tx_ + CY[r] * ty_);
      const double b = (cn[r] <= 0 ? cn[r] * f[r] : 0.0) - 2.0 * A * (CX[r] * Mx + CY[r] * My) +
                       s - kappa * Tn * cn[r];
      ne.row(kr, b);
    }
    double x[5];
    ne.solve(x);
#pragma unroll
    for (int c = 0; c < 3; ++c) f[uq[c]] = x[c];
  }
  double r = 0, Ux = 0, Uy = 0, sxx = 0, sxy = 0, syy = 0, Tt = 0, qx = 0, qy = 0;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const double wf = WD[q] * f[q];
    r += wf;
    Ux += CX[q] * wf;
    Uy += CY[q] * wf;
    sxx += CX[q] * CX[q] * wf;
    sxy += CX[q] * CY[q] * wf;
    syy += CY[q] * CY[q] * wf;
    if constexpr (TH) {
      const double wg = WD[q] * gq[q];
      Tt += wg;
      qx += CX[q] * wg;
      qy += CY[q] * wg;
    }
  }
  mom[0] = r;
  mom[1] = Ux;
  mom[2] = Uy;
  mom[3] = sxx;
  mom[4] = sxy;
  mom[5] = syy;
  mom[6] = Tt;
  mom[7] = qx;
  mom[8] = qy;
}

// Ring nodes without corners, enumerated bottom row, top row, left column,
// right column.
__device__ inline int ring_count(const Geo& g) { return 2 * (g.nx - 2) + 2 * (g.ny - 2); }
__device__ inline void ring_node(const Geo& g, int t, int* i, int* j) {
  const int a = g.nx - 2, b = g.ny - 2;
  if (t < a) { *i = t + 1; *j = 0; }
  else if (t < 2 * a) { *i = t - a + 1; *j = g.ny - 1; }
  else if (t < 2 * a + b) { *i = 0; *j = t - 2 * a + 1; }
  else { *i = g.nx - 1; *j = t - 2 * a - b + 1; }
}
__device__ inline int ring_index(const Geo& g, int i, int j) {
  const int a = g.nx - 2, b = g.ny - 2;
  if (j == 0) return i - 1;
  if (j == g.ny - 1) return a + i - 1;
  if (i == 0) return 2 * a + j - 1;
  return 2 * a + b + j - 1;
}

// Boundary pre-pass of an ALKS step: the least-squares completion of every
// ring node (one thread each), written as raw moments to a perimeter buffer
// that the step kernel reads. Kept apart so that the step kernel does not
// carry the registers of the small dense solves.
template <typename R, bool TH>
__global__ __launch_bounds__(NTHREADS) void alks_ring_kernel(Geo g, AdjArgs<R> a, R* ring) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int nr = ring_count(g);
  if (t >= nr) return;
  int i, j;
  ring_node(g, t, &i, &j);
  const int k = j * g.nx + i;
  double mom[9];
  ring_fill<R, TH>(g, a, i, j, k, a.mask[k], mom);
  constexpr int NM = TH ? 9 : 6;
#pragma unroll
  for (int f = 0; f < NM; ++f) ring[size_t(f) * nr + t] = R(mom[f]);
}

// ---------------------------------------------------------------------------
// ALKS step
// ---------------------------------------------------------------------------
// One ALKS step, adjoint level n+1 -> n. The adjoint state is kept as the
// coefficients of the adjoint equilibria, f~_i^eq = rho~ + c_i.V (eq:afeq)
// and g~_i^eq = Theta (eq:ageq), so a step needs the forward state of one
// level only:
//   stage A  weighted pull of the level-n+1 equilibria from the 8
//            neighbours (eq:ap..eq:aq), or the least-squares completion at
//            ring nodes, for the tile and its halo;
//   stage B  the local terms of eq:albef_ex / eq:albeg_ex at level n
//            (seeds, 3 T q~ coupling, implicit Brinkman
//            u~ = (U~ + T q~ - seed) / (1 + alpha)), then
//            V = 3 u~ + 9 s~ u - 3 rho~ u - 2A div s~ and
//            Theta = T~ + 3 q~.u - B div q~ - grad B . q~ with the
//            level-n state, and the sensitivity
//            3 alpha' u.u~ - B' grad T . q~ (Sec. 2.5).
template <typename R, bool TH>
__global__ __launch_bounds__(NTHREADS) void alks_step_kernel(Geo g, AdjArgs<R> a,
                                                            const R* __restrict__ ring) {
  constexpr int NM = TH ? 9 : 6;
  __shared__ R sm[NM][LPOS];

  int x0, x1, y0, y1;
  tile_extent(blockIdx.x, g.ntx, g.nx, TX, &x0, &x1);
  tile_extent(blockIdx.y, g.nty, g.ny, TY, &y0, &y1);
  const int tw = x1 - x0, th = y1 - y0, hw = tw + 2, hh = th + 2;

  // stage A: raw moments of the pulled (or completed) adjoint populations
  for (int p = threadIdx.x; p < hw * hh; p += NTHREADS) {
    int lx = p % hw, ly = p / hw;
    int i = x0 + lx - 1, j = y0 + ly - 1;
    if (g.periodic) {
      i = wrapi(i, g.nx);
      j = wrapi(j, g.ny);
    } else if (i < 0 || j < 0 || i >= g.nx || j >= g.ny) {
      continue;
    }
    const int k = j * g.nx + i;
    const int pos = ly * LW + lx;
    const int m = a.mask[k];
    const int fc = g.periodic ? FLOW_INTERIOR : (m & 3);
    if (fc == FLOW_CORNER) continue;
    if (fc == FLOW_INTERIOR) {
      R r = R(0), Ux = R(0), Uy = R(0), sxx = R(0), sxy = R(0), syy = R(0);
      R Tt = R(0), qx = R(0), qy = R(0);
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const int iz = g.periodic ? wrapi(i + CX[q], g.nx) : i + CX[q];
        const int jz = g.periodic ? wrapi(j + CY[q], g.ny) : j + CY[q];
        const int kz = jz * g.nx + iz;
        const R E = a.r0[kz] + R(CX[q]) * a.vx0[kz] + R(CY[q]) * a.vy0[kz];
        const R wE = R(WD[q]) * E;
        r += wE;
        if (CX[q]) Ux += R(CX[q]) * wE;
        if (CY[q]) Uy += R(CY[q]) * wE;
        if (CX[q]) sxx += wE;
        if (CX[q] * CY[q]) sxy += R(CX[q] * CY[q]) * wE;
        if (CY[q]) syy += wE;
        if constexpr (TH) {
          const R wT = R(WD[q]) * a.th0[kz];
          Tt += wT;
          if (CX[q]) qx += R(CX[q]) * wT;
          if (CY[q]) qy += R(CY[q]) * wT;
        }
      }
      sm[0][pos] = r;
      sm[1][pos] = Ux;
      sm[2][pos] = Uy;
      sm[3][pos] = sxx;
      sm[4][pos] = sxy;
      sm[5][pos] = syy;
      if constexpr (TH) {
        sm[6][pos] = Tt;
        sm[7][pos] = qx;
        sm[8][pos] = qy;
      }
    } else {
      const int nr = ring_count(g), t = ring_index(g, i, j);
#pragma unroll
      for (int f = 0; f < NM; ++f) sm[f][pos] = ring[size_t(f) * nr + t];
    }
  }
  __syncthreads();
  // corners copy the moments of their y-neighbour (always inside tile+halo)
  if (!g.periodic) {
    for (int p = threadIdx.x; p < hw * hh; p += NTHREADS) {
      int lx = p % hw, ly = p / hw;
      int i = x0 + lx - 1, j = y0 + ly - 1;
      if ((i != 0 && i != g.nx - 1) || (j != 0 && j != g.ny - 1)) continue;
      const int pos = ly * LW + lx;
      const int pn = pos + (j == 0 ? LW : -LW);
#pragma unroll
      for (int f = 0; f < NM; ++f) sm[f][pos] = sm[f][pn];
    }
    __syncthreads();
  }

  // stage B
  const R A2 = R(2.0 * g.A);
  for (int p = threadIdx.x; p < tw * th; p += NTHREADS) {
    const int lx = p % tw, ly = p / tw;
    const int i = x0 + lx, j = y0 + ly;
    const int k = j * g.nx + i;
    const int pos = (ly + 1) * LW + (lx + 1);
    const bool ring = !g.periodic && (i == 0 || j == 0 || i == g.nx - 1 || j == g.ny - 1);
    const bool corner = ring && (i == 0 || i == g.nx - 1) && (j == 0 || j == g.ny - 1);
    // local terms are those of the node whose moments were taken
    const int kl = corner ? (j == 0 ? g.nx + i : (g.ny - 2) * g.nx + i) : k;
    const int ml = a.mask[kl];
    const R r = sm[0][pos];
    R Ux = sm[1][pos], Uy = sm[2][pos];
    const R sxx = sm[3][pos], sxy = sm[4][pos], syy = sm[5][pos];
    R Tt = R(0), qx = R(0), qy = R(0);
    if constexpr (TH) {
      Tt = sm[6][pos];
      qx = sm[7][pos];
      qy = sm[8][pos];
      const R Tl = a.T[kl];
      Ux += Tl * qx;
      Uy += Tl * qy;
      if (ml & TAG_PROBE) {
        Ux -= R(a.seed_heat / 3.0) * Tl;
        Tt -= R(a.seed_heat) * a.ux[kl];
      }
    }
    const R s = a.inv1pa[k];
    const R utx = Ux * s, uty = Uy * s;
    const R ux = a.ux[k], uy = a.uy[k];
    // div s~: (d_x s~xx + d_y s~xy, d_x s~xy + d_y s~yy) from LDS
    auto ldx = [&](int f) {
      return fd_axis<R>(i, g.nx, g.periodic, [&](int o) { return sm[f][pos + o]; });
    };
    auto ldy = [&](int f) {
      return fd_axis<R>(j, g.ny, g.periodic, [&](int o) { return sm[f][pos + o * LW]; });
    };
    const R dsx = ldx(3) + ldy(4);
    const R dsy = ldx(4) + ldy(5);
    const R Vx = R(3) * utx + R(9) * (sxx * ux + sxy * uy) - R(3) * r * ux - A2 * dsx;
    const R Vy = R(3) * uty + R(9) * (sxy * ux + syy * uy) - R(3) * r * uy - A2 * dsy;
    a.r1[k] = r;
    a.vx1[k] = Vx;
    a.vy1[k] = Vy;
    R Th = R(0);
    if constexpr (TH) {
      const R divq = ldx(7) + ldy(8);
      const R Bk = a.B[k];
      const R dBx = gdx(a.B, i, j, g), dBy = gdy(a.B, i, j, g);
      Th = Tt + R(3) * (qx * ux + qy * uy) - Bk * divq - (dBx * qx + dBy * qy);
      a.th1[k] = Th;
    }
    if (a.sens_mode) {
      double v = 0.0;
      if (!ring) {
        v = double(a.dA3[k]) * (double(ux) * double(utx) + double(uy) * double(uty));
        if constexpr (TH) {
          const double dTx = double(gdx(a.T, i, j, g)), dTy = double(gdy(a.T, i, j, g));
          v -= double(a.dB[k]) * (dTx * double(qx) + dTy * double(qy));
        }
      }
      if (a.sens_mode == 1) a.sens[k] += v;
      else a.sens[k] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------
// sum over inlet nodes minus sum over outlet nodes of drho (ring only)
template <typename R>
__global__ __launch_bounds__(NTHREADS) void pressure_drop_kernel(Geo g, const uint8_t* mask,
                                                                const R* d, double* out) {
  __shared__ double red[NTHREADS / 64];
  const int per = 2 * g.nx + 2 * g.ny;
  double part = 0.0;
  for (int t = threadIdx.x; t < per; t += NTHREADS) {
    int i, j;
    if (t < g.nx) { i = t; j = 0; }
    else if (t < 2 * g.nx) { i = t - g.nx; j = g.ny - 1; }
    else if (t < 2 * g.nx + g.ny) { i = 0; j = t - 2 * g.nx; }
    else { i = g.nx - 1; j = t - 2 * g.nx - g.ny; }
    // corners appear twice in this enumeration; they carry no tags
    const int k = j * g.nx + i;
    const int m = mask[k];
    if ((m & 3) == FLOW_CORNER) continue;
    if (m & TAG_J_INLET) part += double(d[k]);
    if (m & TAG_J_OUTLET) part -= double(d[k]);
  }
  double s = block_sum(part, red);
  if (threadIdx.x == 0) *out = s;
}

// sum of u_x T over the probe nodes of the heat objective
template <typename R>
__global__ __launch_bounds__(NTHREADS) void probe_heat_kernel(Geo g, const uint8_t* mask,
                                                             const R* ux, const R* T,
                                                             double* out) {
  __shared__ double red[NTHREADS / 64];
  double part = 0.0;
  for (int k = threadIdx.x; k < g.N; k += NTHREADS)
    if (mask[k] & TAG_PROBE) part += double(ux[k]) * double(T[k]);
  double s = block_sum(part, red);
  if (threadIdx.x == 0) *out = s;
}

__global__ __launch_bounds__(NTHREADS) void sum_kernel(const double* v, int n, double* out) {
  __shared__ double red[NTHREADS / 64];
  double part = 0.0;
  for (int t = threadIdx.x; t < n; t += NTHREADS) part += v[t];
  double s = block_sum(part, red);
  if (threadIdx.x == 0) *out = s;
}

__global__ void fill_kernel(double* p, size_t n, double v) {
  size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}
template <typename R>
__global__ void fill_r_kernel(R* p, size_t n) {
  size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k < n) p[k] = R(0);
}
template <typename R>
__global__ void to_double_kernel(const R* s, double* d, size_t n) {
  size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k < n) d[k] = double(s[k]);
}
template <typename R>
__global__ void from_double_kernel(const double* s, R* d, size_t n) {
  size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k < n) d[k] = R(s[k]);
}
template <typename R>
__global__ void finite_kernel(const R* a, size_t n, int* flag) {
  size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k < n && !isfinite(double(a[k]))) *flag = 1;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(size_t n) { return unsigned((n + 255) / 256); }

template <typename R>
void launch_coef(const Geo& g, const double* gamma, double amax, double qa, double Kf,
                 double Ks, double qk, R* inv1pa, R* B, R* dA3, R* dB, hipStream_t s) {
  coef_kernel<R><<<blocks_for(g.N), 256, 0, s>>>(g, gamma, amax, qa, Kf, Ks, qk, inv1pa, B, dA3,
                                                 dB);
}
template <typename R>
void launch_init(const Geo& g, const uint8_t* mask, const R* ubx, const R* uby, const R* Tb,
                 double fac0, R* d, R* ux, R* uy, R* T, hipStream_t s) {
  init_kernel<R><<<blocks_for(g.N), 256, 0, s>>>(g, mask, ubx, uby, Tb, fac0, d, ux, uy, T);
}
template <typename R>
void launch_lks_step(const Geo& g, const FwdArgs<R>& a, hipStream_t s) {
  dim3 grid(g.ntx, g.nty);
  if (g.thermal) lks_step_kernel<R, true><<<grid, NTHREADS, 0, s>>>(g, a);
  else lks_step_kernel<R, false><<<grid, NTHREADS, 0, s>>>(g, a);
}
template <typename R>
void launch_alks_step(const Geo& g, const AdjArgs<R>& a, R* ring, hipStream_t s) {
  dim3 grid(g.ntx, g.nty);
  if (!g.periodic) {
    const int nr = 2 * (g.nx - 2) + 2 * (g.ny - 2);
    const unsigned nb = unsigned((nr + NTHREADS - 1) / NTHREADS);
    if (g.thermal) alks_ring_kernel<R, true><<<nb, NTHREADS, 0, s>>>(g, a, ring);
    else alks_ring_kernel<R, false><<<nb, NTHREADS, 0, s>>>(g, a, ring);
  }
  if (g.thermal) alks_step_kernel<R, true><<<grid, NTHREADS, 0, s>>>(g, a, ring);
  else alks_step_kernel<R, false><<<grid, NTHREADS, 0, s>>>(g, a, ring);
}
template <typename R>
void launch_pressure_drop(const Geo& g, const uint8_t* mask, const R* d, double* out,
                          hipStream_t s) {
  pressure_drop_kernel<R><<<1, NTHREADS, 0, s>>>(g, mask, d, out);
}
template <typename R>
void launch_probe_heat(const Geo& g, const uint8_t* mask, const R* ux, const R* T, double* out,
                       hipStream_t s) {
  probe_heat_kernel<R><<<1, NTHREADS, 0, s>>>(g, mask, ux, T, out);
}
void launch_sum(const double* v, int n, double* out, hipStream_t s) {
  sum_kernel<<<1, NTHREADS, 0, s>>>(v, n, out);
}
void launch_fill(double* p, size_t n, double v, hipStream_t s) {
  if (n) fill_kernel<<<blocks_for(n), 256, 0, s>>>(p, n, v);
}
template <typename R>
void launch_fill_r(R* p, size_t n, hipStream_t s) {
  if (n) fill_r_kernel<R><<<blocks_for(n), 256, 0, s>>>(p, n);
}
template <typename R>
void launch_to_double(const R* src, double* dst, size_t n, hipStream_t s) {
  to_double_kernel<R><<<blocks_for(n), 256, 0, s>>>(src, dst, n);
}
template <typename R>
void launch_from_double(const double* src, R* dst, size_t n, hipStream_t s) {
  from_double_kernel<R><<<blocks_for(n), 256, 0, s>>>(src, dst, n);
}
template <typename R>
void launch_finite_check(const R* a, size_t n, int* flag, hipStream_t s) {
  finite_kernel<R><<<blocks_for(n), 256, 0, s>>>(a, n, flag);
}

#define LKS_INSTANTIATE(R)                                                                    \
  template void launch_coef<R>(const Geo&, const double*, double, double, double, double,     \
                               double, R*, R*, R*, R*, hipStream_t);                          \
  template void launch_init<R>(const Geo&, const uint8_t*, const R*, const R*, const R*,      \
                               double, R*, R*, R*, R*, hipStream_t);                          \
  template void launch_lks_step<R>(const Geo&, const FwdArgs<R>&, hipStream_t);               \
  template void launch_alks_step<R>(const Geo&, const AdjArgs<R>&, R*, hipStream_t);          \
  template void launch_pressure_drop<R>(const Geo&, const uint8_t*, const R*, double*,        \
                                        hipStream_t);                                         \
  template void launch_probe_heat<R>(const Geo&, const uint8_t*, const R*, const R*, double*,  \
                                     hipStream_t);                                            \
  template void launch_fill_r<R>(R*, size_t, hipStream_t);                                    \
  template void launch_to_double<R>(const R*, double*, size_t, hipStream_t);                  \
  template void launch_from_double<R>(const double*, R*, size_t, hipStream_t);                \
  template void launch_finite_check<R>(const R*, size_t, int*, hipStream_t);

LKS_INSTANTIATE(float)
LKS_INSTANTIATE(double)

}  // namespace lks
