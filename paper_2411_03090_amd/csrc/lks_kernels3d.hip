// D3Q19 kernels: the LKS step and the ALKS step of the three-dimensional
// extension (the equations of Sec. 2.3-2.5 with indices running over x, y,
// z, Sec. 2.1), on gfx950.
//
// Each step is two node-parallel passes with the neighbour gathers served by
// the L1/L2 caches:
//   forward  pass 1  per node the coefficients of f_i^eq and g_i^eq,
//                    f'_i^eq = w_i [a0 + 3 c.u + c.P.c], g_i^eq = w_i [T + c.G]
//                    with a0 = drho - 3/2 u.u, P = 9/2 u u + A (grad u +
//                    grad u^T), G = 3 T u + B grad T (eq:feq2, eq:geq2);
//            pass 2  per node the pull of the 19 equilibria from x - c_i,
//                    the implicit Brinkman division and the face closures;
//   adjoint  pass 1  per node the pull of f~_i^eq = rho~ + c_i.V and
//                    g~_i^eq = Theta from x + c_i (eq:afeq, eq:ageq), the face
//                    least-squares completion, the local terms and the moments
//                    rho~, u~, s~, T~, q~;
//            pass 2  per node V and Theta of the new level from the moments
//                    and the sensitivity 3 alpha' u.u~ - B' grad T.q~.
// Blocks are mapped so that each XCD works on a contiguous slab of nodes,
// keeping the neighbour planes of a block in that XCD's L2.
#include <hip/hip_runtime.h>

#include "lks_device.h"

namespace lks {
namespace {

__device__ constexpr int QX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
__device__ constexpr int QY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
__device__ constexpr int QZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
__device__ constexpr double QW[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                                      1.0 / 18, 1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                      1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                      1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
// symmetric index of (a, b) into xx xy xz yy yz zz
__device__ constexpr int SI[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};

constexpr int NT3 = 256;
constexpr int FLOW_VELOCITY3 = 1;
constexpr int THERM_DIRICHLET3 = 1;
constexpr int TAG_J_INLET3 = 16, TAG_J_OUTLET3 = 32, TAG_PROBE3 = 64, TAG_SOLID3 = 128;

// node of this thread: the blocks of XCD x (blockIdx % 8) cover the x-th
// eighth of the node range
__device__ inline int node3(int N) {
  const int per = int(gridDim.x) / NXCD;
  const int lb = (int(blockIdx.x) % NXCD) * per + int(blockIdx.x) / NXCD;
  const int k = lb * NT3 + int(threadIdx.x);
  return k < N ? k : -1;
}
__device__ inline int logical_block() {
  const int per = int(gridDim.x) / NXCD;
  return (int(blockIdx.x) % NXCD) * per + int(blockIdx.x) / NXCD;
}

struct P3 {
  int i, j, l;
};
__device__ inline P3 decode(const Geo3& g, int k) {
  const int t = k / g.nx;
  return {k - t * g.nx, t % g.ny, t / g.ny};
}
__device__ inline int wrapc(int x, int n) { return x < 0 ? x + n : (x >= n ? x - n : x); }
// node at p + d; periodic axes wrap, the caller never steps past the end of
// a non-periodic axis
__device__ inline int nbr(const Geo3& g, P3 p, int dx, int dy, int dz) {
  int a = p.i + dx, b = p.j + dy, c = p.l + dz;
  if (g.periodic & 1) a = wrapc(a, g.nx);
  if (g.periodic & 2) b = wrapc(b, g.ny);
  if (g.periodic & 4) c = wrapc(c, g.nz);
  return (c * g.ny + b) * g.nx + a;
}
// coordinates at an end of a non-periodic axis; *o = 2 axis + (at the high
// end) of the last one found
__device__ inline int ends(const Geo3& g, P3 p, int* o) {
  int c = 0;
  *o = -1;
  if (!(g.periodic & 1)) {
    if (p.i == 0) { ++c; *o = 0; }
    else if (p.i == g.nx - 1) { ++c; *o = 1; }
  }
  if (!(g.periodic & 2)) {
    if (p.j == 0) { ++c; *o = 2; }
    else if (p.j == g.ny - 1) { ++c; *o = 3; }
  }
  if (!(g.periodic & 4)) {
    if (p.l == 0) { ++c; *o = 4; }
    else if (p.l == g.nz - 1) { ++c; *o = 5; }
  }
  return c;
}
// the node an edge or corner node copies from: inwards along y and z
__device__ inline P3 copy_src(const Geo3& g, P3 p) {
  P3 s = p;
  if (!(g.periodic & 2)) s.j = p.j == 0 ? 1 : (p.j == g.ny - 1 ? g.ny - 2 : p.j);
  if (!(g.periodic & 4)) s.l = p.l == 0 ? 1 : (p.l == g.nz - 1 ? g.nz - 2 : p.l);
  return s;
}

// derivative along axis ax: central inside or across a periodic axis,
// second-order one-sided at the ends of a non-periodic axis
template <typename R>
__device__ inline R dd(const Geo3& g, const R* f, P3 p, int k, int ax) {
  int c, n, per, step;
  if (ax == 0) { c = p.i; n = g.nx; per = g.periodic & 1; step = 1; }
  else if (ax == 1) { c = p.j; n = g.ny; per = g.periodic & 2; step = g.nx; }
  else { c = p.l; n = g.nz; per = g.periodic & 4; step = g.nx * g.ny; }
  if (c > 0 && c < n - 1) return R(0.5) * (f[k + step] - f[k - step]);
  if (per) {
    const int kp = c == n - 1 ? k - (n - 1) * step : k + step;
    const int km = c == 0 ? k + (n - 1) * step : k - step;
    return R(0.5) * (f[kp] - f[km]);
  }
  if (c == 0) return R(0.5) * (R(-3) * f[k] + R(4) * f[k + step] - f[k + 2 * step]);
  return R(0.5) * (R(3) * f[k] - R(4) * f[k - step] + f[k - 2 * step]);
}

__device__ inline double block_sum3(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int w = int(threadIdx.x) / 64, lane = int(threadIdx.x) % 64;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < NT3 / 64; ++i) s += red[i];
  return s;
}

// ---------------------------------------------------------------------------
// design coefficients and initial state
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(NT3) void coef3_kernel(Geo3 g, const uint8_t* __restrict__ mask,
                                                    const double* __restrict__ gamma, double amax,
                                                    double qa, double Kf, double Ks, double qk,
                                                    R* inv1pa, R* B, R* dA3, R* dB) {
  const int k = node3(g.N);
  if (k < 0) return;
  int o;
  if (ends(g, decode(g, k), &o)) {
    inv1pa[k] = R(1);
    B[k] = R(3.0 * (1.0 / 6.0 - Kf));
    dA3[k] = R(0);
    dB[k] = R(0);
    return;
  }
  const double gm = gamma[k];
  const double alpha = amax * qa * (1.0 - gm) / (qa + gm);
  const double dalpha = -amax * qa * (1.0 + qa) / ((qa + gm) * (qa + gm));
  const double K = Kf + (Ks - Kf) * qk * (1.0 - gm) / (qk + gm);
  const double dK = -(Ks - Kf) * qk * (1.0 + qk) / ((qk + gm) * (qk + gm));
  const bool solid = mask[k] & TAG_SOLID3;
  inv1pa[k] = R(1.0 / (1.0 + alpha));
  B[k] = R(3.0 * (1.0 / 6.0 - K));
  dA3[k] = solid ? R(0) : R(3.0 * dalpha);
  dB[k] = solid ? R(0) : R(-3.0 * dK);
}

template <typename R>
__global__ __launch_bounds__(NT3) void init3_kernel(Geo3 g, const uint8_t* __restrict__ mask,
                                                    const R* ubx, const R* uby, const R* ubz,
                                                    const R* Tb, double f0, R* d, R* ux, R* uy,
                                                    R* uz, R* T) {
  const int k = node3(g.N);
  if (k < 0) return;
  const P3 p = decode(g, k);
  int o;
  const int ne = ends(g, p, &o);
  const int m = mask[k];
  d[k] = R(0);
  const bool vel = ne == 1 && (m & 3) == FLOW_VELOCITY3;
  ux[k] = vel ? R(double(ubx[k]) * f0) : R(0);
  uy[k] = vel ? R(double(uby[k]) * f0) : R(0);
  uz[k] = vel ? R(double(ubz[k]) * f0) : R(0);
  if (g.thermal) {
    int kt = k;
    if (ne >= 2) {
      const P3 s = copy_src(g, p);
      kt = (s.l * g.ny + s.j) * g.nx + s.i;
    }
    T[k] = ((mask[kt] >> 2) & 3) == THERM_DIRICHLET3 ? Tb[kt] : R(0);
  }
}

// ---------------------------------------------------------------------------
// LKS step
// ---------------------------------------------------------------------------
template <typename R, bool TH>
__global__ __launch_bounds__(NT3) void eq3_kernel(Geo3 g, Fwd3Args<R> a) {
  const int k = node3(g.N);
  if (k < 0) return;
  const P3 p = decode(g, k);
  const size_t N = size_t(g.N);
  const R* uf[3] = {a.s0[1], a.s0[2], a.s0[3]};
  R u[3], G[3][3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    u[c] = uf[c][k];
#pragma unroll
    for (int b = 0; b < 3; ++b) G[c][b] = dd(g, uf[c], p, k, b);
  }
  const R A = R(g.A);
  const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  R* e = a.e;
  e[k] = a.s0[0][k] - R(1.5) * uu;
#pragma unroll
  for (int x = 0; x < 3; ++x)
#pragma unroll
    for (int y = x; y < 3; ++y)
      e[(1 + SI[x][y]) * N + k] = R(4.5) * u[x] * u[y] + A * (G[x][y] + G[y][x]);
  if constexpr (TH) {
    const R T = a.s0[4][k], Bk = a.B[k];
#pragma unroll
    for (int c = 0; c < 3; ++c)
      e[(7 + c) * N + k] = R(3) * T * u[c] + Bk * dd(g, a.s0[4], p, k, c);
  }
}

// new-level values of a node that is not an edge or corner node
template <typename R, bool TH>
__device__ void lks3_node(const Geo3& g, const Fwd3Args<R>& a, P3 p, int k, int ne, int o,
                          R& d_out, R u_out[3], R& T_out) {
  const size_t N = size_t(g.N);
  const R* e = a.e;
  const int ax = o >> 1, sg = (o & 1) ? 1 : -1;
  R rho = R(0), U[3] = {R(0), R(0), R(0)}, Ts = R(0);
  R S0 = R(0), Sp = R(0), S0g = R(0), Spg = R(0);
#pragma unroll
  for (int q = 0; q < 19; ++q) {
    const int cq[3] = {QX[q], QY[q], QZ[q]};
    int cn = 0;
    if (ne) cn = sg * (ax == 0 ? cq[0] : (ax == 1 ? cq[1] : cq[2]));
    if (cn < 0) continue;
    const int z = nbr(g, p, -cq[0], -cq[1], -cq[2]);
    R cu = R(0), cpc = R(0);
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      if (!cq[x]) continue;
      cu += R(cq[x]) * a.s0[1 + x][z];
      cpc += e[(1 + SI[x][x]) * N + z];
#pragma unroll
      for (int y = x + 1; y < 3; ++y)
        if (cq[y]) cpc += R(2 * cq[x] * cq[y]) * e[(1 + SI[x][y]) * N + z];
    }
    const R f = R(QW[q]) * (e[z] + R(3) * cu + cpc);
    rho += f;
#pragma unroll
    for (int x = 0; x < 3; ++x)
      if (cq[x]) U[x] += R(cq[x]) * f;
    R gq = R(0);
    if constexpr (TH) {
      R cg = R(0);
#pragma unroll
      for (int x = 0; x < 3; ++x)
        if (cq[x]) cg += R(cq[x]) * e[(7 + x) * N + z];
      gq = R(QW[q]) * (a.s0[4][z] + cg);
      Ts += gq;
    }
    if (ne) {
      if (cn == 0) { S0 += f; S0g += gq; }
      else { Sp += f; Spg += gq; }
    }
  }
  const int m = a.mask[k];
  if (!ne) {
    const R s = a.inv1pa[k];
    d_out = rho;
#pragma unroll
    for (int x = 0; x < 3; ++x) u_out[x] = U[x] * s;
    if constexpr (TH) T_out = ((m >> 2) & 3) == THERM_DIRICHLET3 ? a.Tb[k] : Ts;
    return;
  }
  R un;
  if ((m & 3) == FLOW_VELOCITY3) {
    const double fac = a.ufac[a.level_out];
#pragma unroll
    for (int x = 0; x < 3; ++x) u_out[x] = R(double(a.ub[x][k]) * fac);
    un = R(sg) * (ax == 0 ? u_out[0] : (ax == 1 ? u_out[1] : u_out[2]));
    d_out = S0 + R(2) * Sp - un;
  } else {
    const R dro = R(g.drho_out);
    d_out = dro;
    un = S0 + R(2) * Sp - dro;
#pragma unroll
    for (int x = 0; x < 3; ++x) u_out[x] = x == ax ? R(sg) * un : R(0);
  }
  if constexpr (TH) {
    if (((m >> 2) & 3) == THERM_DIRICHLET3) T_out = a.Tb[k];
    else T_out = (S0g + R(2) * Spg) / (R(1) + un);
  }
}

template <typename R, bool TH>
__global__ __launch_bounds__(NT3) void lks3_kernel(Geo3 g, Fwd3Args<R> a) {
  __shared__ double red[NT3 / 64];
  const int k = node3(g.N);
  double part = 0.0;
  if (k >= 0) {
    const P3 p = decode(g, k);
    int o;
    const int ne = ends(g, p, &o);
    R d, u[3], T = R(0);
    if (ne >= 2) {
      const P3 s = copy_src(g, p);
      int os;
      const int nes = ends(g, s, &os);
      lks3_node<R, TH>(g, a, s, (s.l * g.ny + s.j) * g.nx + s.i, nes, os, d, u, T);
      u[0] = u[1] = u[2] = R(0);
    } else {
      lks3_node<R, TH>(g, a, p, k, ne, o, d, u, T);
    }
    a.s1[0][k] = d;
    a.s1[1][k] = u[0];
    a.s1[2][k] = u[1];
    a.s1[3][k] = u[2];
    if constexpr (TH) a.s1[4][k] = T;
    if (a.acc) {
      const int m = a.mask[k];
      if (a.objective == 1) {
        if (m & TAG_PROBE3) part = double(u[0]) * double(T);
      } else {
        if (m & TAG_J_INLET3) part += double(d);
        if (m & TAG_J_OUTLET3) part -= double(d);
      }
    }
  }
  if (a.acc) {
    const double s = block_sum3(part, red);
    if (threadIdx.x == 0) a.acc[logical_block()] += s;
  }
}

// ---------------------------------------------------------------------------
// ALKS step
// ---------------------------------------------------------------------------
template <typename R, bool TH>
__device__ void alks3_node(const Geo3& g, const Adj3Args<R>& a, P3 p, int k, int ne, int o,
                           R mom[14]) {
  const int ax = o >> 1, sg = (o & 1) ? 1 : -1;
  const int m = a.mask[k];
  R f[19], gq[19];
#pragma unroll
  for (int q = 0; q < 19; ++q) {
    const int cq[3] = {QX[q], QY[q], QZ[q]};
    int cn = 0;
    if (ne) cn = sg * (ax == 0 ? cq[0] : (ax == 1 ? cq[1] : cq[2]));
    f[q] = R(0);
    gq[q] = R(0);
    if (cn > 0) continue;
    const int z = nbr(g, p, cq[0], cq[1], cq[2]);
    R v = a.p0[0][z];
#pragma unroll
    for (int x = 0; x < 3; ++x)
      if (cq[x]) v += R(cq[x]) * a.p0[1 + x][z];
    f[q] = v;
    if constexpr (TH) gq[q] = a.p0[4][z];
  }
  R r = R(0), U[3] = {R(0), R(0), R(0)}, S[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
  R Tt = R(0), qv[3] = {R(0), R(0), R(0)};
#pragma unroll
  for (int q = 0; q < 19; ++q) {
    const int cq[3] = {QX[q], QY[q], QZ[q]};
    const R wf = R(QW[q]) * f[q];
    r += wf;
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      if (!cq[x]) continue;
      U[x] += R(cq[x]) * wf;
#pragma unroll
      for (int y = x; y < 3; ++y)
        if (cq[y]) S[SI[x][y]] += R(cq[x] * cq[y]) * wf;
    }
    if constexpr (TH) {
      const R wg = R(QW[q]) * gq[q];
      Tt += wg;
#pragma unroll
      for (int x = 0; x < 3; ++x)
        if (cq[x]) qv[x] += R(cq[x]) * wg;
    }
  }
  const R Tn = TH ? a.T[k] : R(0);
  if (ne) {
    const FaceOp3& op = a.ops[o];
    R kappa = R(0), gu[5] = {R(0), R(0), R(0), R(0), R(0)};
    if constexpr (TH) {
      if (((m >> 2) & 3) == THERM_DIRICHLET3) {
#pragma nounroll
        for (int c = 0; c < 5; ++c) {
          R t = R(0);
#pragma unroll
          for (int q = 0; q < 19; ++q) t += R(op.Ld[c][q]) * gq[q];
          gu[c] = t;
        }
      } else {
        const R* un_src = ax == 0 ? a.u[0] : (ax == 1 ? a.u[1] : a.u[2]);
        const R un = R(sg) * un_src[k];
        R num = R(0);
#pragma unroll
        for (int q = 0; q < 19; ++q) num += (R(op.ga[q]) - un * R(op.ge[q])) * gq[q];
        const R den = R(op.A0) - R(2) * un * R(op.A1) + un * un * R(op.A2);
        kappa = -num / den;
#pragma nounroll
        for (int c = 0; c < 5; ++c) {
          R t = R(0);
#pragma unroll
          for (int q = 0; q < 19; ++q) t += R(op.Lg0[c][q]) * gq[q];
          gu[c] = t - kappa * (R(op.hc[c]) - un * R(op.h1[c]));
        }
      }
    }
    R s = R(0);
    if (m & TAG_J_INLET3) s += R(a.seed_dp / 3.0);
    if (m & TAG_J_OUTLET3) s -= R(a.seed_dp / 3.0);
    const int v = (m & 3) == FLOW_VELOCITY3 ? 0 : 1;
    const R kT = kappa * Tn;
#pragma nounroll
    for (int c = 0; c < 5; ++c) {
      R t = R(op.Ls[v][c]) * s + R(op.Lk[v][c]) * kT;
#pragma unroll
      for (int q = 0; q < 19; ++q) t += R(op.Lf[v][c][q]) * f[q];
      const R wf = R(op.uw[c]) * t;
      const R cx[3] = {R(op.uc[c][0]), R(op.uc[c][1]), R(op.uc[c][2])};
      r += wf;
#pragma unroll
      for (int x = 0; x < 3; ++x) {
        U[x] += cx[x] * wf;
#pragma unroll
        for (int y = x; y < 3; ++y) S[SI[x][y]] += cx[x] * cx[y] * wf;
      }
      if constexpr (TH) {
        const R wg = R(op.uw[c]) * gu[c];
        Tt += wg;
#pragma unroll
        for (int x = 0; x < 3; ++x) qv[x] += cx[x] * wg;
      }
    }
  }
  if constexpr (TH) {
    const bool probe = (m & TAG_PROBE3) && a.seed_heat != 0.0;
    if (probe) Tt -= R(a.seed_heat) * a.u[0][k];
    if (!ne && ((m >> 2) & 3) == THERM_DIRICHLET3) {
      Tt = R(0);
      qv[0] = qv[1] = qv[2] = R(0);
    }
#pragma unroll
    for (int x = 0; x < 3; ++x) U[x] += Tn * qv[x];
    if (probe) U[0] -= R(a.seed_heat / 3.0) * Tn;
  }
  const R s = a.inv1pa[k];
  mom[0] = r;
#pragma unroll
  for (int x = 0; x < 3; ++x) mom[1 + x] = U[x] * s;
#pragma unroll
  for (int c = 0; c < 6; ++c) mom[4 + c] = S[c];
  mom[10] = Tt;
#pragma unroll
  for (int x = 0; x < 3; ++x) mom[11 + x] = qv[x];
}

template <typename R, bool TH>
__global__ __launch_bounds__(NT3) void alks3_pull_kernel(Geo3 g, Adj3Args<R> a) {
  const int k = node3(g.N);
  if (k < 0) return;
  const P3 p = decode(g, k);
  int o;
  const int ne = ends(g, p, &o);
  R mom[14];
  if (ne >= 2) {
    const P3 s = copy_src(g, p);
    int os;
    const int nes = ends(g, s, &os);
    alks3_node<R, TH>(g, a, s, (s.l * g.ny + s.j) * g.nx + s.i, nes, os, mom);
  } else {
    alks3_node<R, TH>(g, a, p, k, ne, o, mom);
  }
  const size_t N = size_t(g.N);
  constexpr int NM = TH ? 14 : 10;
#pragma unroll
  for (int c = 0; c < NM; ++c) a.m[c * N + k] = mom[c];
}

template <typename R, bool TH>
__global__ __launch_bounds__(NT3) void alks3_eq_kernel(Geo3 g, Adj3Args<R> a) {
  const int k = node3(g.N);
  if (k < 0) return;
  const P3 p = decode(g, k);
  const size_t N = size_t(g.N);
  const R* M = a.m;
  const R u[3] = {a.u[0][k], a.u[1][k], a.u[2][k]};
  const R r = M[k];
  const R A2 = R(2.0 * g.A);
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    R su = R(0), ds = R(0);
#pragma unroll
    for (int y = 0; y < 3; ++y) {
      const R* sf = M + (4 + SI[x][y]) * N;
      su += sf[k] * u[y];
      ds += dd(g, sf, p, k, y);
    }
    a.p1[1 + x][k] = R(3) * M[(1 + x) * N + k] + R(9) * su - R(3) * r * u[x] - A2 * ds;
  }
  a.p1[0][k] = r;
  R qv[3] = {R(0), R(0), R(0)};
  if constexpr (TH) {
    R qu = R(0), divq = R(0), gbq = R(0);
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      qv[x] = M[(11 + x) * N + k];
      qu += qv[x] * u[x];
      divq += dd(g, M + (11 + x) * N, p, k, x);
      gbq += dd(g, a.B, p, k, x) * qv[x];
    }
    a.p1[4][k] = M[10 * N + k] + R(3) * qu - a.B[k] * divq - gbq;
  }
  if (a.sens_mode) {
    int o;
    double v = 0.0;
    if (!ends(g, p, &o) && !(a.mask[k] & TAG_SOLID3)) {
      double uu = 0.0;
#pragma unroll
      for (int x = 0; x < 3; ++x) uu += double(u[x]) * double(M[(1 + x) * N + k]);
      v = double(a.dA3[k]) * uu;
      if constexpr (TH) {
        double gq = 0.0;
#pragma unroll
        for (int x = 0; x < 3; ++x) gq += double(dd(g, a.T, p, k, x)) * double(qv[x]);
        v -= double(a.dB[k]) * gq;
      }
    }
    if (a.sens_mode == 1) a.sens[k] += v;
    else a.sens[k] = v;
  }
}

// objective sum over tagged nodes (steady runs): pressure-drop tags of
// drho, or the probe enthalpy flux u_x T; one block, fixed order
template <typename R>
__global__ __launch_bounds__(NT3) void tag_sum3_kernel(Geo3 g, const uint8_t* __restrict__ mask,
                                                       const R* d, const R* ux, const R* T,
                                                       int objective, double* out) {
  __shared__ double red[NT3 / 64];
  double s = 0.0;
  for (int k = int(threadIdx.x); k < g.N; k += NT3) {
    const int m = mask[k];
    if (objective == 1) {
      if (m & TAG_PROBE3) s += double(ux[k]) * double(T[k]);
    } else {
      if (m & TAG_J_INLET3) s += double(d[k]);
      if (m & TAG_J_OUTLET3) s -= double(d[k]);
    }
  }
  s = block_sum3(s, red);
  if (threadIdx.x == 0) out[0] = s;
}

}  // namespace

int blocks3(int N) {
  const int b = (N + NT3 - 1) / NT3;
  return NXCD * ((b + NXCD - 1) / NXCD);
}

template <typename R>
void launch_coef3(const Geo3& g, const uint8_t* mask, const double* gamma, double alpha_max,
                  double q_alpha, double Kf, double Ks, double qK, R* inv1pa, R* B, R* dA3,
                  R* dB, hipStream_t s) {
  coef3_kernel<R><<<blocks3(g.N), NT3, 0, s>>>(g, mask, gamma, alpha_max, q_alpha, Kf, Ks, qK,
                                               inv1pa, B, dA3, dB);
}

template <typename R>
void launch_init3(const Geo3& g, const uint8_t* mask, const R* const ub[3], const R* Tb,
                  double ufac0, R* const st[5], hipStream_t s) {
  init3_kernel<R><<<blocks3(g.N), NT3, 0, s>>>(g, mask, ub[0], ub[1], ub[2], Tb, ufac0, st[0],
                                               st[1], st[2], st[3], st[4]);
}

template <typename R>
void launch_lks3_step(const Geo3& g, const Fwd3Args<R>& a, hipStream_t s) {
  const unsigned nb = unsigned(blocks3(g.N));
  if (g.thermal) {
    eq3_kernel<R, true><<<nb, NT3, 0, s>>>(g, a);
    lks3_kernel<R, true><<<nb, NT3, 0, s>>>(g, a);
  } else {
    eq3_kernel<R, false><<<nb, NT3, 0, s>>>(g, a);
    lks3_kernel<R, false><<<nb, NT3, 0, s>>>(g, a);
  }
}

template <typename R>
void launch_alks3_step(const Geo3& g, const Adj3Args<R>& a, hipStream_t s) {
  const unsigned nb = unsigned(blocks3(g.N));
  if (g.thermal) {
    alks3_pull_kernel<R, true><<<nb, NT3, 0, s>>>(g, a);
    alks3_eq_kernel<R, true><<<nb, NT3, 0, s>>>(g, a);
  } else {
    alks3_pull_kernel<R, false><<<nb, NT3, 0, s>>>(g, a);
    alks3_eq_kernel<R, false><<<nb, NT3, 0, s>>>(g, a);
  }
}

template <typename R>
void launch_tag_sum3(const Geo3& g, const uint8_t* mask, const R* d, const R* ux, const R* T,
                     int objective, double* out, hipStream_t s) {
  tag_sum3_kernel<R><<<1, NT3, 0, s>>>(g, mask, d, ux, T, objective, out);
}

#define LKS3_INSTANTIATE(R)                                                                   \
  template void launch_coef3<R>(const Geo3&, const uint8_t*, const double*, double, double,  \
                                double, double, double, R*, R*, R*, R*, hipStream_t);        \
  template void launch_init3<R>(const Geo3&, const uint8_t*, const R* const[3], const R*,    \
                                double, R* const[5], hipStream_t);                           \
  template void launch_lks3_step<R>(const Geo3&, const Fwd3Args<R>&, hipStream_t);           \
  template void launch_alks3_step<R>(const Geo3&, const Adj3Args<R>&, hipStream_t);          \
  template void launch_tag_sum3<R>(const Geo3&, const uint8_t*, const R*, const R*, const R*, \
                                   int, double*, hipStream_t);
LKS3_INSTANTIATE(float)
LKS3_INSTANTIATE(double)

}  // namespace lks
