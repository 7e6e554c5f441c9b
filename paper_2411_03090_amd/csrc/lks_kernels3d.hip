// D3Q19 kernels: the LKS step and the ALKS step of the three-dimensional
// extension (the equations of Sec. 2.3-2.5 with indices running over x, y,
// z, Sec. 2.1), on gfx950.
//
// LKS step: one z-marching kernel. A block owns 64 x 4 columns and walks
// through a range of z-planes with the state of two planes in LDS; per plane
// it forms a0 = drho - 3/2 u.u, P = 9/2 u u + A (grad u + grad u^T),
// G = 3 T u + B grad T and the equilibria f'_i^eq = w_i [a0 + 3 c.u + c.P.c],
// g_i^eq = w_i [T + c.G] (eq:feq2, eq:geq2) of the tile and its ring, streams
// them to the columns that pull them, and closes the plane behind with the
// implicit Brinkman division and the face closures. Edge and corner nodes
// are copied by a small second kernel.
// ALKS step: two passes.
//   pass 1  node-parallel: the pull of f~_i^eq = rho~ + c_i.V and
//           g~_i^eq = Theta from x + c_i (eq:afeq, eq:ageq) through L1/L2,
//           the face least-squares completion, the local terms and the
//           moments rho~, u~, s~, T~, q~, stored to a scratch;
//   pass 2  z-marching: V and Theta of the new level from the moments and
//           the sensitivity 3 alpha' u.u~ - B' grad T.q~.
// Blocks are mapped so that each XCD works on a contiguous slab of nodes,
// keeping the neighbour planes of a block in that XCD's L2.
#include <hip/hip_runtime.h>

#include <climits>
#include <vector>

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
// z-marching tiles
// ---------------------------------------------------------------------------
// A block owns a tile of ZX x ZY columns and marches through a range of
// z-planes. Each iteration loads one plane of the inputs (the tile plus a
// 2-node halo, rows coalesced) into LDS, so a field plane leaves HBM once per
// block and every neighbour gather reads LDS. The last tile along x or y is
// shifted to end at the domain end (its overlap with the previous tile is
// computed but not written), so one-sided differences at the ends stay
// inside the tile.
constexpr int ZX = 64, ZY = 4, ZT = ZX * ZY;
constexpr int SX = ZX + 4, NSR = SX * (ZY + 4);    // tile + 2-node halo
constexpr int CXN = ZX + 2, NCR = CXN * (ZY + 2);  // tile + 1-node halo
constexpr int SRL = (NSR + ZT - 1) / ZT;           // halo-region loads per thread
static_assert(ZT == NT3, "one block size for the 3D kernels");
// the directions with an x or y component: their values cross columns
__device__ constexpr int LQ[16] = {1, 2, 3, 4, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18};

__host__ __device__ inline int zchunks(const Geo3& g) {
  const int zc = g.zc < 2 ? 2 : g.zc;
  return g.nz / zc > 1 ? g.nz / zc : 1;
}
__host__ __device__ inline int ztiles(int n, int t) { return (n + t - 1) / t; }

struct ZTile {
  int x0, y0, w, h;  // origin and extent of the tile
  int xo, yo;        // first column and row the block writes
  int z0, z1;        // output planes
  int lb;            // logical block
};

// tile of this block; logical blocks run x fastest, then y, then z-chunk, and
// the blocks of XCD x (blockIdx % 8) take the x-th eighth of them
// (output planes: chunks of [zlo, zhi), nch of them when given)
__device__ inline bool ztile(const Geo3& g, ZTile& t, int zlo = 0, int zhi = -1, int nch = 0) {
  if (zhi < 0) zhi = g.nz;
  if (nch <= 0) nch = zchunks(g);
  const int ntx = ztiles(g.nx, ZX), nty = ztiles(g.ny, ZY);
  const int per = int(gridDim.x) / NXCD;
  t.lb = (int(blockIdx.x) % NXCD) * per + int(blockIdx.x) / NXCD;
  if (t.lb >= ntx * nty * nch) return false;
  const int ix = t.lb % ntx, iy = (t.lb / ntx) % nty, ic = t.lb / (ntx * nty);
  t.w = g.nx < ZX ? g.nx : ZX;
  t.h = g.ny < ZY ? g.ny : ZY;
  t.xo = ix * ZX;
  t.yo = iy * ZY;
  t.x0 = t.xo < g.nx - t.w ? t.xo : g.nx - t.w;
  t.y0 = t.yo < g.ny - t.h ? t.yo : g.ny - t.h;
  t.z0 = zlo + int((long long)ic * (zhi - zlo) / nch);
  t.z1 = zlo + int((long long)(ic + 1) * (zhi - zlo) / nch);
  return true;
}

// coordinate c of an axis of n nodes, wrapped on a periodic axis, -1 beyond a
// non-periodic one (c is at most 2 nodes outside, and n >= 3)
__device__ inline int axc(int c, int n, int per) {
  if (c < 0) return per ? c + n : -1;
  if (c >= n) return per ? c - n : -1;
  return c;
}
// -1 / +1 at the low / high end of a non-periodic axis, else 0
__device__ inline int endof(int c, int n, int per) {
  return per ? 0 : (c == 0 ? -1 : (c == n - 1 ? 1 : 0));
}
__device__ inline int zwrap(int s, int n) { return s < 0 ? s + n : (s >= n ? s - n : s); }

// a column of the tile or of its 1-node ring
struct ZNode {
  int on;      // the thread has this column
  int dx, dy;  // tile-local position, -1 .. w and -1 .. h
  int lds;     // index in the 2-node halo region
  int ci;      // index in the 1-node halo region
  int off;     // in-plane offset j nx + i, -1 off the domain
  int ex, ey;  // end flags of the column
};

__device__ inline ZNode znode(const Geo3& g, const ZTile& t, int dx, int dy, bool on) {
  ZNode n;
  n.on = on;
  n.dx = dx;
  n.dy = dy;
  n.lds = (dy + 2) * SX + dx + 2;
  n.ci = (dy + 1) * CXN + dx + 1;
  const int x = axc(t.x0 + dx, g.nx, g.periodic & 1), y = axc(t.y0 + dy, g.ny, g.periodic & 2);
  n.off = (x < 0 || y < 0) ? -1 : y * g.nx + x;
  n.ex = x < 0 ? 0 : endof(x, g.nx, g.periodic & 1);
  n.ey = y < 0 ? 0 : endof(y, g.ny, g.periodic & 2);
  return n;
}

// the ring column at position r of the ring around the tile: the row below
// the tile, the row above, the column left of it, the column right of it
__device__ inline ZNode zring_at(const Geo3& g, const ZTile& t, int r) {
  const int a = t.w + 2;
  int dx, dy;
  if (r < a) {
    dx = r - 1;
    dy = -1;
  } else if (r < 2 * a) {
    dx = r - a - 1;
    dy = t.h;
  } else if (r < 2 * a + t.h) {
    dx = -1;
    dy = r - 2 * a;
  } else {
    dx = t.w;
    dy = r - 2 * a - t.h;
  }
  const bool on = r >= 0 && r < 2 * a + 2 * t.h;
  return znode(g, t, on ? dx : 0, on ? dy : 0, on);
}
// the thread's ring column: three of the four waves take a third of the ring
// each, in consecutive positions (neighbouring lanes touch neighbouring LDS
// words); the wave left out rotates with the block, so that over the blocks
// resident on a CU the ring work is spread evenly over the SIMDs, and a wave
// runs the ring code only where it holds ring columns
__device__ inline ZNode zring(const Geo3& g, const ZTile& t) {
  const int per = (2 * (t.w + 2) + 2 * t.h + 2) / 3;  // at most 47 for 64 x 4 tiles
  const int lane = int(threadIdx.x) % 64, w = int(threadIdx.x) / 64;
  const int k = (w - (t.lb & 3) + 4) & 3;  // 0: the wave without ring columns
  return zring_at(g, t, (k > 0 && lane < per) ? (k - 1) * per + lane : -1);
}

// in-plane offsets of the thread's elements of the 2-node halo region; -1
// off the domain or beyond the tile's region
__device__ inline void zregion(const Geo3& g, const ZTile& t, int off[SRL]) {
#pragma unroll
  for (int r = 0; r < SRL; ++r) {
    const int e = int(threadIdx.x) + r * ZT;
    const int dx = e % SX - 2, dy = e / SX - 2;
    off[r] = -1;
    if (e < NSR && dx < t.w + 2 && dy < t.h + 2) {
      const int x = axc(t.x0 + dx, g.nx, g.periodic & 1);
      const int y = axc(t.y0 + dy, g.ny, g.periodic & 2);
      if (x >= 0 && y >= 0) off[r] = y * g.nx + x;
    }
  }
}

// one plane of NF fields over the thread's region elements (zero where the
// plane or the node does not exist)
// (SEL: elements off the domain or of a missing plane load the field's first
// node and keep zero, with no per-element branches; the LKS step gains by it,
// the ALKS march, whose loads wait longer, does not)
template <typename R, int NF, bool SEL = false>
__device__ inline void zload(const R* const F[NF], bool exists, unsigned base, const int off[SRL],
                             R v[SRL][NF]) {
#pragma unroll
  for (int r = 0; r < SRL; ++r) {
    const bool in = exists && off[r] >= 0;
    if constexpr (SEL) {
      const unsigned o = in ? base + unsigned(off[r]) : 0u;
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const R x = F[f][o];
        v[r][f] = in ? x : R(0);
      }
    } else {
#pragma unroll
      for (int f = 0; f < NF; ++f) v[r][f] = in ? F[f][base + unsigned(off[r])] : R(0);
    }
  }
}
template <typename R, int NF>
__device__ inline void zstore(R (*dst)[NSR], const R v[SRL][NF]) {
#pragma unroll
  for (int r = 0; r < SRL; ++r) {
    const int e = int(threadIdx.x) + r * ZT;
    if (e < NSR)
#pragma unroll
      for (int f = 0; f < NF; ++f) dst[f][e] = v[r][f];
  }
}

// difference at index i of an LDS field along a stride st: central, or
// second-order one-sided at the low (e < 0) or high (e > 0) end of an axis
template <typename R>
__device__ inline R d1(const R* f, int i, int st, int e) {
  if (e == 0) return R(0.5) * (f[i + st] - f[i - st]);
  if (e < 0) return R(0.5) * (R(-3) * f[i] + R(4) * f[i + st] - f[i + 2 * st]);
  return R(0.5) * (R(3) * f[i] - R(4) * f[i - st] + f[i - 2 * st]);
}
// d1 of the product f * h
template <typename R>
__device__ inline R d1p(const R* f, const R* h, int i, int st, int e) {
  auto at = [&](int o) { return f[i + o * st] * h[i + o * st]; };
  if (e == 0) return R(0.5) * (at(1) - at(-1));
  if (e < 0) return R(0.5) * (R(-3) * at(0) + R(4) * at(1) - at(2));
  return R(0.5) * (R(3) * at(0) - R(4) * at(-1) + at(-2));
}

// ---------------------------------------------------------------------------
// LKS step
// ---------------------------------------------------------------------------
// Per plane s of the march, every column of the tile and its ring forms the
// coefficients a0 = drho - 3/2 u.u, P = 9/2 u u + A (grad u + grad u^T),
// G = 3 T u + B grad T and the 19 equilibria f'_q = w_q [a0 + 3 c.u + c.P.c],
// g_q = w_q [T + c.G] of its node (eq:feq2, eq:geq2). The values with an x or
// y component go through LDS to the column they stream to; every column adds
// what it receives from plane s to the moments of planes s - 1, s, s + 1 that
// it keeps in registers (the pull of f_i^eq(x - c_i)). Plane s - 1 is then
// complete. A source off the domain sends zeros, so a face node's sums over
// the directions it receives are rho + sg (c_n . f) with n its normal.
template <typename R, bool TH>
struct FwdZLds {
  R st[2][TH ? 4 : 3][NSR];  // u (3), T of planes s and s + 1
  R fq[16][ZT];              // f'_q arriving at each column
  // T and G = 3 T u + B grad T of every column of the tile and its ring (1-node
  // halo region): a column forms the g_q = w_q (T + c_q.G) it receives itself
  R tg[TH ? 4 : 1][TH ? NCR : 1];
  double red[ZT / 64];
};

// moments of three planes (s - 1, s, s + 1) of a column
template <typename R, bool TH>
struct FwdAcc {
  R r[3], U[3][3], T[3], Q[3][3];
};

template <typename R, bool TH>
__device__ inline void facc_add(FwdAcc<R, TH>& A, int q, R f, R gv) {
  const int sl = QZ[q] + 1;
  A.r[sl] += f;
  if (QX[q]) A.U[sl][0] += R(QX[q]) * f;
  if (QY[q]) A.U[sl][1] += R(QY[q]) * f;
  if (QZ[q]) A.U[sl][2] += R(QZ[q]) * f;
  if constexpr (TH) {
    A.T[sl] += gv;
    if (QX[q]) A.Q[sl][0] += R(QX[q]) * gv;
    if (QY[q]) A.Q[sl][1] += R(QY[q]) * gv;
    if (QZ[q]) A.Q[sl][2] += R(QZ[q]) * gv;
  }
}

template <typename R, bool TH>
__device__ inline void facc_shift(FwdAcc<R, TH>& A) {
  A.r[0] = A.r[1];
  A.r[1] = A.r[2];
  A.r[2] = R(0);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    A.U[0][c] = A.U[1][c];
    A.U[1][c] = A.U[2][c];
    A.U[2][c] = R(0);
  }
  if constexpr (TH) {
    A.T[0] = A.T[1];
    A.T[1] = A.T[2];
    A.T[2] = R(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      A.Q[0][c] = A.Q[1][c];
      A.Q[1][c] = A.Q[2][c];
      A.Q[2][c] = R(0);
    }
  }
}

// z difference of a field at plane s from its values at s - 1 (zp), s (fc)
// and s + 1 (zn); z2 is plane 2 (low end) or nz - 3 (high end)
template <typename R>
__device__ inline R dz3(int ez, R fc, R zp, R zn, R z2) {
  if (ez < 0) return R(0.5) * (R(-3) * fc + R(4) * zn - z2);
  if (ez > 0) return R(0.5) * (R(3) * fc - R(4) * zp + z2);
  return R(0.5) * (zn - zp);
}

// equilibria of the node of column n at plane sw, sent to the columns they
// stream to; the own column keeps its c = 0 and c = +-e_z values. zp holds
// u and T of plane sw - 1 and is advanced to plane sw.
template <typename R, bool TH, bool OWN>
__device__ inline void fwd_src(const Geo3& g, const Fwd3Args<R>& a, FwdZLds<R, TH>& L,
                               const ZTile& t, const ZNode& n, int cur, int nxt, bool hn, int sw,
                               unsigned nxy, R dk, R Bk, R zp[4], FwdAcc<R, TH>& A) {
  if (!n.on) return;
  R fv[19], gv[19];
  R tgv[4] = {R(0), R(0), R(0), R(0)};
  if (n.off < 0) {
#pragma unroll
    for (int q = 0; q < 19; ++q) fv[q] = gv[q] = R(0);
  } else {
    const int i = n.lds;
    const int ez = endof(sw, g.nz, g.periodic & 4);
    R u[3], zn[4] = {R(0), R(0), R(0), R(0)}, z2[4] = {R(0), R(0), R(0), R(0)};
    constexpr int NZ = TH ? 4 : 3;
#pragma unroll
    for (int c = 0; c < 3; ++c) u[c] = L.st[cur][c][i];
    const R T = TH ? L.st[cur][TH ? 3 : 0][i] : R(0);
    if (hn)
#pragma unroll
      for (int c = 0; c < NZ; ++c) zn[c] = L.st[nxt][c][i];
    if (ez) {
      const unsigned b2 = unsigned(ez < 0 ? 2 : g.nz - 3) * nxy + unsigned(n.off);
#pragma unroll
      for (int c = 0; c < NZ; ++c) z2[c] = a.s0[1 + c][b2];
    }
    R G[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      G[c][0] = d1(L.st[cur][c], i, 1, n.ex);
      G[c][1] = d1(L.st[cur][c], i, SX, n.ey);
      G[c][2] = dz3(ez, u[c], zp[c], zn[c], z2[c]);
    }
    const R A_ = R(g.A);
    const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const R a0 = dk - R(1.5) * uu;
    R P[6];
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
      for (int y = x; y < 3; ++y) P[SI[x][y]] = R(4.5) * u[x] * u[y] + A_ * (G[x][y] + G[y][x]);
    R Gt[3] = {R(0), R(0), R(0)};
    if constexpr (TH) {
      const R dT[3] = {d1(L.st[cur][TH ? 3 : 0], i, 1, n.ex), d1(L.st[cur][TH ? 3 : 0], i, SX, n.ey),
                       dz3(ez, T, zp[3], zn[3], z2[3])};
#pragma unroll
      for (int c = 0; c < 3; ++c) Gt[c] = R(3) * T * u[c] + Bk * dT[c];
      zp[3] = T;
      tgv[0] = T;
#pragma unroll
      for (int c = 0; c < 3; ++c) tgv[1 + c] = Gt[c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) zp[c] = u[c];
#pragma unroll
    for (int q = 0; q < 19; ++q) {
      const int cq[3] = {QX[q], QY[q], QZ[q]};
      R cu = R(0), cpc = R(0), cg = R(0);
#pragma unroll
      for (int x = 0; x < 3; ++x) {
        if (!cq[x]) continue;
        cu += R(cq[x]) * u[x];
        cpc += P[SI[x][x]];
#pragma unroll
        for (int y = x + 1; y < 3; ++y)
          if (cq[y]) cpc += R(2 * cq[x] * cq[y]) * P[SI[x][y]];
        if constexpr (TH) cg += R(cq[x]) * Gt[x];
      }
      fv[q] = R(QW[q]) * (a0 + R(3) * cu + cpc);
      gv[q] = TH ? R(QW[q]) * (T + cg) : R(0);
    }
  }
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int q = LQ[j];
    const int px = n.dx + QX[q], py = n.dy + QY[q];
    if (px >= 0 && px < t.w && py >= 0 && py < t.h) {
      L.fq[j][py * ZX + px] = fv[q];
    }
  }
  if constexpr (TH)
#pragma unroll
    for (int c = 0; c < 4; ++c) L.tg[c][n.ci] = tgv[c];
  if constexpr (OWN) {
    facc_add(A, 0, fv[0], gv[0]);
    facc_add(A, 5, fv[5], gv[5]);
    facc_add(A, 6, fv[6], gv[6]);
  }
}

// component ax of (v0, v1, v2)
template <typename R>
__device__ inline R pick3(int ax, R v0, R v1, R v2) {
  return (ax == 0 ? v0 : R(0)) + (ax == 1 ? v1 : R(0)) + (ax == 2 ? v2 : R(0));
}

// new-level values of a node from its moments: the implicit Brinkman
// division inside, the velocity / pressure closures and the temperature
// closure on faces; edge and corner nodes are copied afterwards
template <typename R, bool TH>
__device__ inline void fwd3_out(const Geo3& g, const Fwd3Args<R>& a, unsigned k, int ex, int ey,
                                int ez, int m, R s, R Tb, const R ubk[3], double fac, R rho,
                                const R U[3], R Ts, const R Q[3], double& part) {
  const int ne = (ex != 0) + (ey != 0) + (ez != 0);
  if (ne >= 2) return;
  R d, u[3], T = R(0);
  if (!ne) {
    d = rho;
#pragma unroll
    for (int x = 0; x < 3; ++x) u[x] = U[x] * s;
    if constexpr (TH) T = ((m >> 2) & 3) == THERM_DIRICHLET3 ? Tb : Ts;
  } else {
    const int ax = ex ? 0 : (ey ? 1 : 2);
    const int sg = ex ? ex : (ey ? ey : ez);
    // components along the normal as masked sums (no indexing by ax, which
    // would move the register arrays to memory)
    const R Un = pick3(ax, U[0], U[1], U[2]);
    const R sn = rho + R(sg) * Un;  // S0 + 2 S+ over the received directions
    R un;
    if ((m & 3) == FLOW_VELOCITY3) {
#pragma unroll
      for (int x = 0; x < 3; ++x) u[x] = R(double(ubk[x]) * fac);
      un = R(sg) * pick3(ax, u[0], u[1], u[2]);
      d = sn - un;
    } else {
      const R dro = R(g.drho_out);
      d = dro;
      un = sn - dro;
#pragma unroll
      for (int x = 0; x < 3; ++x) u[x] = x == ax ? R(sg) * un : R(0);
    }
    if constexpr (TH) {
      const R Qn = pick3(ax, Q[0], Q[1], Q[2]);
      if (((m >> 2) & 3) == THERM_DIRICHLET3) T = Tb;
      // heat-flux face: Tb holds the flux qbar into the domain (0: adiabatic)
      else T = (Ts + R(sg) * Qn + Tb) / (R(1) + un);
    }
  }
  a.s1[0][k] = d;
  a.s1[1][k] = u[0];
  a.s1[2][k] = u[1];
  a.s1[3][k] = u[2];
  if constexpr (TH) a.s1[4][k] = T;
  if (a.acc) {
    if (a.objective == 1) {
      if (m & TAG_PROBE3) part += double(u[0]) * double(T);
    } else {
      if (m & TAG_J_INLET3) part += double(d);
      if (m & TAG_J_OUTLET3) part -= double(d);
    }
  }
}

template <typename R, bool TH>
__global__ __launch_bounds__(ZT) void lks3z_kernel(Geo3 g, Fwd3Args<R> a) {
  constexpr int NF = TH ? 4 : 3;  // u (3), T in the LDS ring
  __shared__ FwdZLds<R, TH> L;
  ZTile t;
  if (!ztile(g, t)) return;
  const int tid = int(threadIdx.x), lx = tid % ZX, ly = tid / ZX;
  const int pz = g.periodic & 4;
  const unsigned nxy = unsigned(g.nx) * unsigned(g.ny);
  int roff[SRL];
  zregion(g, t, roff);
  const ZNode n0 = znode(g, t, lx, ly, lx < t.w && ly < t.h);
  const ZNode n1 = zring(g, t);
  const bool own = n0.on && t.x0 + lx >= t.xo && t.y0 + ly >= t.yo;
  // source planes: one beyond the output range on each side where it exists
  const int sb = (t.z0 == 0 && !pz) ? 0 : t.z0 - 1;
  const int se = (t.z1 == g.nz && !pz) ? g.nz - 1 : t.z1;
  const R* F[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) F[f] = a.s0[1 + f];
  R v[SRL][NF];
  zload<R, NF, true>(F, true, unsigned(zwrap(sb, g.nz)) * nxy, roff, v);
  zstore<R, NF>(L.st[0], v);
  auto has = [&](int s) { return pz || (s >= 0 && s < g.nz); };
  if (has(sb + 1)) zload<R, NF, true>(F, true, unsigned(zwrap(sb + 1, g.nz)) * nxy, roff, v);
  R zp0[4] = {R(0), R(0), R(0), R(0)}, zp1[4] = {R(0), R(0), R(0), R(0)};
  if (has(sb - 1)) {
    const unsigned b = unsigned(zwrap(sb - 1, g.nz)) * nxy;
#pragma unroll
    for (int c = 0; c < NF; ++c) {
      if (n0.on && n0.off >= 0) zp0[c] = F[c][b + unsigned(n0.off)];
      if (n1.on && n1.off >= 0) zp1[c] = F[c][b + unsigned(n1.off)];
    }
  }
  // per-node inputs one iteration ahead: drho and B of the source nodes,
  // class, Brinkman factor and prescribed temperature of the output node
  // the prescribed velocity of a velocity face node is read with the rest,
  // a plane ahead, and the level's inflow factor once
  const double fac = a.ufac[a.level_out];
  auto node_in = [&](int s, R& d0, R& d1_, R& b0, R& b1, int& mk, R& ip, R& tb, R ub[3]) {
    d0 = d1_ = b0 = b1 = ip = tb = R(0);
    ub[0] = ub[1] = ub[2] = R(0);
    mk = 0;
    if (!has(s)) return;
    const unsigned base = unsigned(zwrap(s, g.nz)) * nxy;
    if (n0.on && n0.off >= 0) {
      d0 = a.s0[0][base + unsigned(n0.off)];
      if constexpr (TH) b0 = a.B[base + unsigned(n0.off)];
    }
    if (n1.on && n1.off >= 0) {
      d1_ = a.s0[0][base + unsigned(n1.off)];
      if constexpr (TH) b1 = a.B[base + unsigned(n1.off)];
    }
    const int p = s - 1;
    if (own && p >= t.z0 && p < t.z1) {
      const unsigned k = unsigned(p) * nxy + unsigned(n0.off);
      mk = a.mask[k];
      ip = a.inv1pa[k];
      if constexpr (TH) tb = a.Tb[k];
      if (n0.ex || n0.ey || endof(p, g.nz, pz))  // a face node (not waiting for its class)
#pragma unroll
        for (int x = 0; x < 3; ++x) ub[x] = a.ub[x][k];
    }
  };
  R dd0, dd1, b0, b1, ip, tb, ub[3];
  int mk;
  node_in(sb, dd0, dd1, b0, b1, mk, ip, tb, ub);
  FwdAcc<R, TH> A = {};
  double part = 0.0;
  for (int s = sb; s <= se; ++s) {
    const int it = s - sb, cur = it & 1, nxt = cur ^ 1;
    const bool hn = has(s + 1);
    if (hn) zstore<R, NF>(L.st[nxt], v);
    lds_barrier();
    if (has(s + 2)) zload<R, NF, true>(F, true, unsigned(zwrap(s + 2, g.nz)) * nxy, roff, v);
    const R cd0 = dd0, cd1 = dd1, cb0 = b0, cb1 = b1, cip = ip, ctb = tb;
    const R cub[3] = {ub[0], ub[1], ub[2]};
    const int cmk = mk;
    if (s + 1 <= se) node_in(s + 1, dd0, dd1, b0, b1, mk, ip, tb, ub);
    const int sw = zwrap(s, g.nz);
    fwd_src<R, TH, true>(g, a, L, t, n0, cur, nxt, hn, sw, nxy, cd0, cb0, zp0, A);
    fwd_src<R, TH, false>(g, a, L, t, n1, cur, nxt, hn, sw, nxy, cd1, cb1, zp1, A);
    lds_barrier();
    if (n0.on) {
      const int me = ly * ZX + lx;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int q = LQ[j];
        R gv = R(0);
        if constexpr (TH) {
          // g_q of the source column x - c_q, summed as at the source
          const int src = (ly - QY[q] + 1) * CXN + (lx - QX[q] + 1);
          const int cq[3] = {QX[q], QY[q], QZ[q]};
          R cg = R(0);
#pragma unroll
          for (int x = 0; x < 3; ++x)
            if (cq[x]) cg += R(cq[x]) * L.tg[1 + x][src];
          gv = R(QW[q]) * (L.tg[0][src] + cg);
        }
        facc_add(A, q, L.fq[j][me], gv);
      }
    }
    const int p = s - 1;
    if (own && p >= t.z0 && p < t.z1)
      fwd3_out<R, TH>(g, a, unsigned(p) * nxy + unsigned(n0.off), n0.ex, n0.ey,
                      endof(p, g.nz, pz), cmk, cip, ctb, cub, fac, A.r[0], A.U[0], A.T[0],
                      A.Q[0], part);
    facc_shift(A);
  }
  if (!pz && se == g.nz - 1 && own) {
    const unsigned k = unsigned(g.nz - 1) * nxy + unsigned(n0.off);
    const R ubk[3] = {a.ub[0][k], a.ub[1][k], a.ub[2][k]};
    fwd3_out<R, TH>(g, a, k, n0.ex, n0.ey, 1, a.mask[k], a.inv1pa[k], TH ? a.Tb[k] : R(0), ubk,
                    fac, A.r[0], A.U[0], A.T[0], A.Q[0], part);
  }
  if (a.acc) {
    const double s = block_sum3(part, L.red);
    if (tid == 0) a.acc[t.lb] += s;
  }
}

// edge and corner nodes: density and temperature of the node one step
// inwards along y and z, zero velocity
template <typename R, bool TH>
__global__ __launch_bounds__(NT3) void copy3_kernel(Geo3 g, const int* __restrict__ list, int n,
                                                    R* d, R* ux, R* uy, R* uz, R* T) {
  const int i = int(blockIdx.x) * NT3 + int(threadIdx.x);
  if (i >= n) return;
  const int k = list[i];
  const P3 s = copy_src(g, decode(g, k));
  const int ks = (s.l * g.ny + s.j) * g.nx + s.i;
  d[k] = d[ks];
  ux[k] = R(0);
  uy[k] = R(0);
  uz[k] = R(0);
  if constexpr (TH) T[k] = T[ks];
}

// ---------------------------------------------------------------------------
// ALKS step
// ---------------------------------------------------------------------------
// raw moments of the 19 pulled values f~_q, g~_q, summed by weight class
// (rest, the six axis directions, and the three diagonal planes):
// rho~, u~ (3), s~ xx xy xz yy yz zz, T~, q~ (3)
template <typename R, bool TH>
__device__ inline void mom19(const R f[19], const R g[19], R M[14]) {
  const R w0 = R(1.0 / 3), w1 = R(1.0 / 18), w2 = R(1.0 / 36);
  // axis pairs (1,2) x, (3,4) y, (5,6) z
  const R sa[3] = {f[1] + f[2], f[3] + f[4], f[5] + f[6]};
  const R da[3] = {f[1] - f[2], f[3] - f[4], f[5] - f[6]};
  // diagonal planes xy (7-10), xz (11-14), yz (15-18): directions
  // (+,+), (-,-), (+,-), (-,+) in the plane's two axes
  R ps[3], sab[3], d1[3], d2[3];
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const int q = 7 + 4 * p;
    const R s1 = f[q] + f[q + 1], s2 = f[q + 2] + f[q + 3];
    d1[p] = f[q] - f[q + 1];
    d2[p] = f[q + 2] - f[q + 3];
    ps[p] = s1 + s2;
    sab[p] = s1 - s2;
  }
  M[0] = w0 * f[0] + w1 * (sa[0] + sa[1] + sa[2]) + w2 * (ps[0] + ps[1] + ps[2]);
  M[1] = w1 * da[0] + w2 * ((d1[0] + d2[0]) + (d1[1] + d2[1]));
  M[2] = w1 * da[1] + w2 * ((d1[0] - d2[0]) + (d1[2] + d2[2]));
  M[3] = w1 * da[2] + w2 * ((d1[1] - d2[1]) + (d1[2] - d2[2]));
  M[4] = w1 * sa[0] + w2 * (ps[0] + ps[1]);
  M[5] = w2 * sab[0];
  M[6] = w2 * sab[1];
  M[7] = w1 * sa[1] + w2 * (ps[0] + ps[2]);
  M[8] = w2 * sab[2];
  M[9] = w1 * sa[2] + w2 * (ps[1] + ps[2]);
  if constexpr (TH) {
    const R ga[3] = {g[1] + g[2], g[3] + g[4], g[5] + g[6]};
    const R ha[3] = {g[1] - g[2], g[3] - g[4], g[5] - g[6]};
    R gs[3], e1[3], e2[3];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const int q = 7 + 4 * p;
      gs[p] = (g[q] + g[q + 1]) + (g[q + 2] + g[q + 3]);
      e1[p] = g[q] - g[q + 1];
      e2[p] = g[q + 2] - g[q + 3];
    }
    M[10] = w0 * g[0] + w1 * (ga[0] + ga[1] + ga[2]) + w2 * (gs[0] + gs[1] + gs[2]);
    M[11] = w1 * ha[0] + w2 * ((e1[0] + e2[0]) + (e1[1] + e2[1]));
    M[12] = w1 * ha[1] + w2 * ((e1[0] - e2[0]) + (e1[2] + e2[2]));
    M[13] = w1 * ha[2] + w2 * ((e1[1] - e2[1]) + (e1[2] - e2[2]));
  } else {
    M[10] = M[11] = M[12] = M[13] = R(0);
  }
}

// the fill of face_fill with the operator op of orientation o and flow type
// v (0 velocity, 1 pressure node)
template <typename R, bool TH, typename OP>
__device__ inline void face_apply(OP op, int v, int o, const Adj3Args<R>& a, int k, int m, R Tn,
                                  const R f[19], const R gq[19], R M[14]) {
  const int ax = o >> 1, sg = (o & 1) ? 1 : -1;
  R kappa = R(0), gu[5] = {R(0), R(0), R(0), R(0), R(0)};
  if constexpr (TH) {
    if (((m >> 2) & 3) == THERM_DIRICHLET3) {
#pragma nounroll
      for (int c = 0; c < 5; ++c) {
        R t = R(0);
#pragma unroll
        for (int q = 0; q < 19; ++q) t += op->Ld[c][q] * gq[q];
        gu[c] = t;
      }
    } else {
      const R* un_src = ax == 0 ? a.u[0] : (ax == 1 ? a.u[1] : a.u[2]);
      const R un = R(sg) * un_src[k];
      R num = R(0);
#pragma unroll
      for (int q = 0; q < 19; ++q) num += (op->ga[q] - un * op->ge[q]) * gq[q];
      const R den = op->A0 - R(2) * un * op->A1 + un * un * op->A2;
      kappa = -num / den;
#pragma nounroll
      for (int c = 0; c < 5; ++c) {
        R t = R(0);
#pragma unroll
        for (int q = 0; q < 19; ++q) t += op->Lg0[c][q] * gq[q];
        gu[c] = t - kappa * (op->hc[c] - un * op->h1[c]);
      }
    }
  }
  // boundary seed of the pressure-drop objective per unit boundary pressure
  R s = R(0);
  if (m & TAG_J_INLET3) s += R(a.seed_dp);
  if (m & TAG_J_OUTLET3) s -= R(a.seed_dp);
  const R kT = kappa * Tn;
#pragma nounroll
  for (int c = 0; c < 5; ++c) {
    R t = op->Ls[v][c] * s + op->Lk[v][c] * kT;
#pragma unroll
    for (int q = 0; q < 19; ++q) t += op->Lf[v][c][q] * f[q];
    const R wf = op->uw[c] * t;
    const R cx[3] = {op->uc[c][0], op->uc[c][1], op->uc[c][2]};
    M[0] += wf;
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      M[1 + x] += cx[x] * wf;
#pragma unroll
      for (int y = x; y < 3; ++y) M[4 + SI[x][y]] += cx[x] * cx[y] * wf;
    }
    if constexpr (TH) {
      const R wg = op->uw[c] * gu[c];
      M[10] += wg;
#pragma unroll
      for (int x = 0; x < 3; ++x) M[11 + x] += cx[x] * wg;
    }
  }
}

// least-squares fill of a face node with orientation o: the moments of its
// five missing directions from the 14 received ones (zero in f, g at the
// missing directions), the J seed and the thermal closure. A wave whose
// lanes share orientation and node type reads the operator through the
// scalar unit; mixed waves read it per lane.
template <typename R, bool TH>
__device__ void face_fill(const Adj3Args<R>& a, int k, int m, int o, R Tn, const R f[19],
                          const R gq[19], R M[14]) {
  const int v = (m & 3) == FLOW_VELOCITY3 ? 0 : 1;
  const int key = 2 * o + v;
  const int uk = __builtin_amdgcn_readfirstlane(key);
  if (__all(key == uk))
    face_apply<R, TH>(as_scalar(a.ops) + (uk >> 1), uk & 1, uk >> 1, a, k, m, Tn, f, gq, M);
  else
    face_apply<R, TH>(a.ops + o, v, o, a, k, m, Tn, f, gq, M);
}

// local terms of the adjoint moments: the probe seed, the prescribed
// temperature inside, the T q~ coupling and the Brinkman factor of u~
template <typename R, bool TH>
__device__ inline void adj_local(const Adj3Args<R>& a, int k, int m, int ne, R Tn, R s,
                                 R M[14], R u0) {
  if constexpr (TH) {
    const bool probe = (m & TAG_PROBE3) && a.seed_heat != 0.0;
    if (probe) M[10] -= R(a.seed_heat) * u0;
    // a prescribed temperature does not depend on the arriving populations:
    // zero thermal adjoint inside (both modes) and on faces (exact mode)
    if (((m >> 2) & 3) == THERM_DIRICHLET3 && (!ne || a.exact)) {
      M[10] = R(0);
      M[11] = M[12] = M[13] = R(0);
    }
#pragma unroll
    for (int x = 0; x < 3; ++x) M[1 + x] += Tn * M[11 + x];
    if (probe) M[1] -= R(a.seed_heat / 3.0) * Tn;
  }
#pragma unroll
  for (int x = 0; x < 3; ++x) M[1 + x] *= s;
}

// moments of the node p (not an edge or corner node) with orientation o if
// it is a face node; FACE = false compiles the interior rule alone (ne = 0)
template <typename R, bool TH, bool FACE = true>
__device__ void alks3_node(const Geo3& g, const Adj3Args<R>& a, P3 p, int k, int ne, int o,
                           R M[14]) {
  if constexpr (!FACE) ne = 0;
  const int ax = o >> 1, sg = (o & 1) ? 1 : -1;
  R f[19], gq[19];
#pragma unroll
  for (int q = 0; q < 19; ++q) {
    const int cq[3] = {QX[q], QY[q], QZ[q]};
    int cn = 0;
    if (FACE && ne) cn = sg * (ax == 0 ? cq[0] : (ax == 1 ? cq[1] : cq[2]));
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
  mom19<R, TH>(f, gq, M);
  const int m = a.mask[k];
  const R Tn = TH ? a.T[k] : R(0);
  if constexpr (FACE)
    if (ne) face_fill<R, TH>(a, k, m, o, Tn, f, gq, M);
  // exact mode: u~ stays undivided; the update pass divides V instead
  const bool probe = TH && (m & TAG_PROBE3) && a.seed_heat != 0.0;
  adj_local<R, TH>(a, k, m, ne, Tn, a.exact ? R(1) : a.inv1pa[k], M, probe ? a.u[0][k] : R(0));
}

// ALKS pass 1 at the interior nodes; the boundary nodes are left to
// alks3_face_kernel, so the face completion does not diverge inside the
// waves of the rows that end on an x face
template <typename R, bool TH>
__global__ __launch_bounds__(NT3) void alks3_pull_kernel(Geo3 g, Adj3Args<R> a) {
  const int k = node3(g.N);
  if (k < 0) return;
  const P3 p = decode(g, k);
  int o;
  if (ends(g, p, &o)) return;
  R mom[14];
  alks3_node<R, TH, false>(g, a, p, k, 0, -1, mom);
  const size_t N = size_t(g.N);
  constexpr int NM = TH ? 14 : 10;
#pragma unroll
  for (int c = 0; c < NM; ++c) a.m[c * N + k] = mom[c];
}

// ALKS pass 1 at the boundary nodes of the host-built list (faces grouped by
// orientation, then edges and corners, which take the moments of the node
// one step inwards along y and z)
template <typename R, bool TH>
__global__ __launch_bounds__(NT3) void alks3_face_kernel(Geo3 g, Adj3Args<R> a) {
  const int t = int(blockIdx.x) * NT3 + int(threadIdx.x);
  if (t >= a.nface) return;
  const int k = a.face[t];
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

// in-plane offsets of the thread's elements of the 1-node halo region; -1
// off the domain or beyond the tile's region
__device__ inline void zregion1(const Geo3& g, const ZTile& t, int off[2]) {
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int e = int(threadIdx.x) + r * ZT;
    const int dx = e % CXN - 1, dy = e / CXN - 1;
    off[r] = -1;
    if (e < NCR && dx < t.w + 1 && dy < t.h + 1) {
      const int x = axc(t.x0 + dx, g.nx, g.periodic & 1);
      const int y = axc(t.y0 + dy, g.ny, g.periodic & 2);
      if (x >= 0 && y >= 0) off[r] = y * g.nx + x;
    }
  }
}

// per-node inputs of the ALKS update at one node: its moments rho~, u~,
// T~, its velocity, the coefficients' derivatives, 1/(1 + alpha) and class
template <typename R>
struct AdjIn {
  R r, U[3], Tt, u[3], dA, dB, ip;
  int mk;
  double so;  // the node's accumulated sensitivity (sens_mode 1), read ahead
};

// The ALKS update at node k of a z-march column (eq:afp - eq:agq): V and
// Theta of the new level from the node's moments (cu), the in-plane moment
// fields E (s~xx s~xy s~xz s~yy s~yz q~x q~y T B, 1-node halo, index ci,
// end flags ex, ey) and the z differences zd of s~xz s~yz s~zz q~z T B (z
// window zc, zm1, zn, z2 for the product difference of the exact mode), and
// the sensitivity 3 alpha' u.u~ - B' grad T.q~ (paper) or its exact-mode
// counterpart.
template <typename R, bool TH>
__device__ inline void adj3_update(const Adj3Args<R>& a, const Geo3& g, unsigned k,
                                   const R (*E)[NCR], int ci, int ex, int ey, int ez,
                                   const AdjIn<R>& cu, const R zd[6], const R zc[6],
                                   const R zm1[6], const R zn[6], const R z2[6]) {
  // no fused multiply-adds here: the fused step passes z differences the
  // compiler could fold into the sums below, the update pass selects them
  // per plane, and both must round alike
#pragma clang fp contract(off)
  const R S[6] = {E[0][ci], E[1][ci], E[2][ci], E[3][ci], E[4][ci], zc[2]};
  const R A2 = R(2.0 * g.A);
  const R ds[3] = {d1(E[0], ci, 1, ex) + d1(E[1], ci, CXN, ey) + zd[0],
                   d1(E[1], ci, 1, ex) + d1(E[3], ci, CXN, ey) + zd[1],
                   d1(E[2], ci, 1, ex) + d1(E[4], ci, CXN, ey) + zd[2]};
  R V[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    R su = R(0);
#pragma unroll
    for (int b = 0; b < 3; ++b) su += S[SI[c][b]] * cu.u[b];
    V[c] = R(3) * cu.U[c] + R(9) * su - R(3) * cu.r * cu.u[c] - A2 * ds[c];
  }
  // the Brinkman pairing of the sensitivity: 3 alpha' u.u~ (paper) or
  // alpha' u.V / (1 + alpha) with the undivided V, which then propagates
  // divided by 1 + alpha (exact)
  double pair = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) pair += double(cu.u[c]) * double(a.exact ? V[c] : cu.U[c]);
  if (a.exact) {
    pair *= double(cu.ip) / 3.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) V[c] *= cu.ip;
  }
  a.p1[0][k] = cu.r;
  a.p1[1][k] = V[0];
  a.p1[2][k] = V[1];
  a.p1[3][k] = V[2];
  R qv[3] = {R(0), R(0), R(0)};
  if constexpr (TH) {
    qv[0] = E[5][ci];
    qv[1] = E[6][ci];
    qv[2] = zc[3];
    const R qu = qv[0] * cu.u[0] + qv[1] * cu.u[1] + qv[2] * cu.u[2];
    const R* Bp = E[8];
    if (a.exact) {
      // exact: the transpose of the forward B c.grad_h T, -div_h (B q~)
      const R zbq = dz3(ez, zc[3] * zc[5], zm1[3] * zm1[5], zn[3] * zn[5], z2[3] * z2[5]);
      const R dbq = d1p(Bp, E[5], ci, 1, ex) + d1p(Bp, E[6], ci, CXN, ey) + zbq;
      a.p1[4][k] = cu.Tt + R(3) * qu - dbq;
    } else {
      const R divq = d1(E[5], ci, 1, ex) + d1(E[6], ci, CXN, ey) + zd[3];
      const R gbq = d1(Bp, ci, 1, ex) * qv[0] + d1(Bp, ci, CXN, ey) * qv[1] + zd[5] * qv[2];
      a.p1[4][k] = cu.Tt + R(3) * qu - Bp[ci] * divq - gbq;
    }
  }
  if (a.sens_mode) {
    double sv = 0.0;
    if (!ex && !ey && !ez && !(cu.mk & TAG_SOLID3)) {
      sv = a.sens_b_only ? 0.0 : double(cu.dA) * pair;
      if constexpr (TH) {
        const R* Tp = E[7];
        const R gt[3] = {d1(Tp, ci, 1, ex), d1(Tp, ci, CXN, ey), zd[4]};
        double gq = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) gq += double(gt[c]) * double(qv[c]);
        sv -= double(cu.dB) * gq;
      }
    }
    // the accumulated value was read with the node's other inputs, a plane
    // ahead, so that the read-modify-write does not wait for it here
    if (a.sens_mode == 1) a.sens[k] = cu.so + sv;
    else a.sens[k] = sv;
  }
}

// ALKS pass 2, z-marching: V, Theta (eq:afp - eq:agq) and the sensitivity
// from the moments; x and y differences from an LDS plane, z differences
// from a window of three planes in registers.
// The update pass. LDS plane fields: s~xx s~xy s~xz s~yy s~yz (q~x q~y T B),
// 1-node halo, two planes.
template <typename R, bool TH>
struct AdjELds {
  static constexpr int NE = TH ? 9 : 5;
  R e[2][NE][NCR];
};

// ENDS: only the two end planes of a non-periodic z axis (after the fused
// step, which leaves them): tile chunk 0 takes plane 0, chunk 1 plane nz - 1
template <typename R, bool TH, bool ENDS = false>
__global__ __launch_bounds__(ZT) void alks3e_kernel(Geo3 g, Adj3Args<R> a) {
  constexpr int NE = AdjELds<R, TH>::NE;
  constexpr int NZ = TH ? 6 : 3;  // z window: s~xz s~yz s~zz (q~z T B)
  __shared__ AdjELds<R, TH> L;
  ZTile t;
  if constexpr (ENDS) {
    if (!ztile(g, t, 0, 2, 2)) return;
    if (t.z0 == 1) {
      t.z0 = g.nz - 1;
      t.z1 = g.nz;
    }
  } else {
    if (!ztile(g, t)) return;
  }
  const int tid = int(threadIdx.x), lx = tid % ZX, ly = tid / ZX;
  const int pz = g.periodic & 4;
  const unsigned nxy = unsigned(g.nx) * unsigned(g.ny);
  const unsigned N = unsigned(g.N);
  int coff[2];
  zregion1(g, t, coff);
  const ZNode n0 = znode(g, t, lx, ly, lx < t.w && ly < t.h);
  const bool own = n0.on && t.x0 + lx >= t.xo && t.y0 + ly >= t.yo;
  // plane fields: moments 4, 5, 6, 7, 8 (11, 12) and T, B
  const R* FE[9];
  FE[0] = a.m + 4 * N;
  FE[1] = a.m + 5 * N;
  FE[2] = a.m + 6 * N;
  FE[3] = a.m + 7 * N;
  FE[4] = a.m + 8 * N;
  FE[5] = a.m + 11 * N;
  FE[6] = a.m + 12 * N;
  FE[7] = a.T;
  FE[8] = a.B;
  // z window fields: moments 6, 8, 9 (13) and T, B
  const R* FZ[6] = {a.m + 6 * N, a.m + 8 * N, a.m + 9 * N, a.m + 13 * N, a.T, a.B};
  auto has = [&](int s) { return pz || (s >= 0 && s < g.nz); };
  R v[2][NE];
  auto load = [&](int s) {
    const bool e = has(s);
    const unsigned b = unsigned(zwrap(s, g.nz)) * nxy;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int f = 0; f < NE; ++f) v[r][f] = (e && coff[r] >= 0) ? FE[f][b + coff[r]] : R(0);
  };
  auto store = [&](int slot) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int e = tid + r * ZT;
      if (e < NCR)
#pragma unroll
        for (int f = 0; f < NE; ++f) L.e[slot][f][e] = v[r][f];
    }
  };
  auto zload = [&](int s, R z[6]) {
#pragma unroll
    for (int f = 0; f < 6; ++f) z[f] = R(0);
    if (!own || !has(s)) return;
    const unsigned k = unsigned(zwrap(s, g.nz)) * nxy + unsigned(n0.off);
#pragma unroll
    for (int f = 0; f < NZ; ++f) z[f] = FZ[f][k];
  };
  // per-node inputs one plane ahead
  using In = AdjIn<R>;
  auto node_in = [&](int p, In& q) {
    q.r = q.Tt = q.dA = q.dB = R(0);
    q.ip = R(1);
    q.mk = 0;
    q.so = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) q.U[c] = q.u[c] = R(0);
    if (!own || p >= t.z1) return;
    const unsigned k = unsigned(p) * nxy + unsigned(n0.off);
    q.r = a.m[k];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      q.U[c] = a.m[(1 + c) * N + k];
      q.u[c] = a.u[c][k];
    }
    if constexpr (TH) q.Tt = a.m[10 * N + k];
    q.mk = a.mask[k];
    if (a.exact) q.ip = a.inv1pa[k];
    if (a.sens_mode) {
      q.dA = a.dA3[k];
      if constexpr (TH) q.dB = a.dB[k];
      if (a.sens_mode == 1) q.so = a.sens[k];
    }
  };
  load(t.z0);
  store(0);
  load(t.z0 + 1);
  R zm1[6], zc[6], zn[6];
  zload(t.z0 - 1, zm1);
  zload(t.z0, zc);
  zload(t.z0 + 1, zn);
  In nx;
  node_in(t.z0, nx);
  const int ci = n0.ci;
  for (int p = t.z0; p < t.z1; ++p) {
    const int it = p - t.z0, sc = it & 1;
    lds_barrier();
    if (p + 1 < t.z1) {
      store(sc ^ 1);
      load(p + 2);
    }
    const In cu = nx;
    node_in(p + 1, nx);
    R znn[6];
    zload(p + 2, znn);  // the window's next plane, in flight during this one
    R z2[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
    const int ez = endof(zwrap(p, g.nz), g.nz, pz);
    if (ez < 0) zload(2, z2);
    if (ez > 0) zload(g.nz - 3, z2);
    R zd[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) zd[f] = dz3(ez, zc[f], zm1[f], zn[f], z2[f]);
    if (own)
      adj3_update<R, TH>(a, g, unsigned(p) * nxy + unsigned(n0.off), L.e[sc], ci, n0.ex, n0.ey,
                         ez, cu, zd, zc, zm1, zn, z2);
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      zm1[f] = zc[f];
      zc[f] = zn[f];
      zn[f] = znn[f];
    }
  }
}

// ---------------------------------------------------------------------------
// ALKS step, fused
// ---------------------------------------------------------------------------
// One z-march per block over the planes 1 .. nz-2 of a non-periodic z axis
// (every plane of a periodic one). At plane s every column of the tile and of
// its 1-node ring forms its moments of plane s: an interior node pulls
// f~_q = rho~ + c_q.V and g~_q = Theta from x + c_q (eq:afeq, eq:ageq) out
// of three LDS plane slots of the level-(n+1) coefficients (tile plus a
// 2-node halo; the next plane waits in registers) and applies the local
// terms, as the pull pass does; a
// boundary node takes the moments the face pass left in the scratch. The
// plane's in-plane moment fields go to LDS, the column keeps its own in
// registers, and plane s - 1 is updated (adj3_update) from the moments of
// planes s - 2, s - 1 and s. The moments that never leave the block are not
// stored; only the z-window moments of planes 1, 2, nz-3 and nz-2 go to the
// scratch, for the end planes that alks3e<ENDS> updates afterwards.
// FP32 keeps three coefficient slots and one plane of moment fields, with
// three barriers per plane (their LDS allows three blocks per CU); FP64, held
// to one block per CU by its registers either way, keeps four slots and two
// moment planes with one barrier per plane
template <typename R, bool TH>
struct AdjFLds {
  static constexpr int NP = TH ? 5 : 4;  // rho~, Vx, Vy, Vz (, Theta)
  static constexpr int NE = TH ? 9 : 5;  // s~xx s~xy s~xz s~yy s~yz (q~x q~y T B)
  static constexpr bool LEAN = sizeof(R) == 4;
  static constexpr int NS = LEAN ? 3 : 4;
  R p[NS][NP][NSR];
  R e[LEAN ? 1 : 2][NE][NCR];
};

// node of a column at one plane: index, class, boundary count, T, B and
// 1/(1 + alpha)
template <typename R>
struct ColIn {
  unsigned k;
  int m, ne, valid;
  R T, B, ip;
};

template <typename R, bool TH>
__global__ __launch_bounds__(ZT) void alks3f_kernel(Geo3 g, Adj3Args<R> a) {
  constexpr int NP = AdjFLds<R, TH>::NP, NS = AdjFLds<R, TH>::NS;
  constexpr bool LEAN = AdjFLds<R, TH>::LEAN;
  constexpr int NM = TH ? 14 : 10;
  __shared__ AdjFLds<R, TH> L;
  const int pz = g.periodic & 4;
  ZTile t;
  if (!ztile(g, t, pz ? 0 : 1, pz ? g.nz : g.nz - 1)) return;
  const int tid = int(threadIdx.x), lx = tid % ZX, ly = tid / ZX;
  const unsigned nxy = unsigned(g.nx) * unsigned(g.ny);
  const size_t N = size_t(g.N);
  int roff[SRL];
  zregion(g, t, roff);
  const ZNode n0 = znode(g, t, lx, ly, lx < t.w && ly < t.h);
  const ZNode n1 = zring(g, t);
  const bool own = n0.on && t.x0 + lx >= t.xo && t.y0 + ly >= t.yo;
  const R* F[NP];
#pragma unroll
  for (int f = 0; f < NP; ++f) F[f] = a.p0[f];
  // planes that exist (INT_MIN: none, to skip a column's inputs)
  auto has = [&](int q) { return q != INT_MIN && (pz || (q >= 0 && q < g.nz)); };
  const int base = t.z0 - 2;  // first plane held in the LDS slots
  auto slot = [&](int q) { return (q - base) % NS; };
  const int last = t.z1 + 1;  // last plane the pulls read
  R v[SRL][NP];
  auto load = [&](int q) {
    zload<R, NP>(F, has(q), unsigned(zwrap(q, g.nz)) * nxy, roff, v);
  };
  auto store = [&](int q) { zstore<R, NP>(L.p[slot(q)], v); };
  auto col_in = [&](const ZNode& n, int q, ColIn<R>& c) {
    c.k = 0;
    c.m = c.ne = c.valid = 0;
    c.T = c.B = c.ip = R(0);
    if (!n.on || n.off < 0 || !has(q)) return;
    const int zq = zwrap(q, g.nz);
    c.k = unsigned(zq) * nxy + unsigned(n.off);
    c.valid = 1;
    c.ne = (n.ex != 0) + (n.ey != 0) + (endof(zq, g.nz, pz) != 0);
    c.m = a.mask[c.k];
    if constexpr (TH) {
      c.T = a.T[c.k];
      c.B = a.B[c.k];
    }
    if (!a.exact && !c.ne) c.ip = a.inv1pa[c.k];
  };
  // the face pass's moments of a boundary node (all NM for the own column,
  // the in-plane fields for a ring column) and the probe's velocity, read at
  // the top of the plane so that their latency hides behind the pulls
  auto bnd_in = [&](const ColIn<R>& c, bool all, R Mb[14], R& u0) {
#pragma unroll
    for (int i = 0; i < 14; ++i) Mb[i] = R(0);
    u0 = R(0);
    if (!c.valid) return;
    if (c.ne) {
#pragma unroll
      for (int i = 0; i < NM; ++i)
        if (all || i == 4 || i == 5 || i == 6 || i == 7 || i == 8 || i == 11 || i == 12)
          Mb[i] = a.m[size_t(i) * N + c.k];
    } else if (TH && (c.m & TAG_PROBE3) && a.seed_heat != 0.0) {
      u0 = a.u[0][c.k];
    }
  };
  // moments of a column's node at plane q
  auto moments = [&](const ZNode& n, const ColIn<R>& c, int q, const R Mb[14], R u0, R M[14]) {
#pragma unroll
    for (int i = 0; i < 14; ++i) M[i] = R(0);
    if (!c.valid) return;
    if (c.ne) {
#pragma unroll
      for (int i = 0; i < 14; ++i) M[i] = Mb[i];
      return;
    }
    const int sl[3] = {slot(q - 1), slot(q), slot(q + 1)};
    R f[19], gq[19];
#pragma unroll
    for (int d = 0; d < 19; ++d) {
      const int o = n.lds + QX[d] + QY[d] * SX;
      const int pl = sl[QZ[d] + 1];
      R x = L.p[pl][0][o];
      if (QX[d]) x += R(QX[d]) * L.p[pl][1][o];
      if (QY[d]) x += R(QY[d]) * L.p[pl][2][o];
      if (QZ[d]) x += R(QZ[d]) * L.p[pl][3][o];
      f[d] = x;
      gq[d] = TH ? L.p[pl][TH ? 4 : 0][o] : R(0);
    }
    mom19<R, TH>(f, gq, M);
    adj_local<R, TH>(a, int(c.k), c.m, 0, c.T, a.exact ? R(1) : c.ip, M, u0);
  };
  auto store_e = [&](const ZNode& n, const R M[14], const ColIn<R>& c, int sl) {
    if (!n.on) return;
    R(*E)[NCR] = L.e[sl];
    E[0][n.ci] = M[4];
    E[1][n.ci] = M[5];
    E[2][n.ci] = M[6];
    E[3][n.ci] = M[7];
    E[4][n.ci] = M[8];
    if constexpr (TH) {
      E[TH ? 5 : 0][n.ci] = M[11];
      E[TH ? 6 : 0][n.ci] = M[12];
      E[TH ? 7 : 0][n.ci] = c.T;
      E[TH ? 8 : 0][n.ci] = c.B;
    }
  };
  // the own node's inputs of the update at plane q
  auto upd_in = [&](int q, AdjIn<R>& u) {
    u.r = u.Tt = u.dA = u.dB = R(0);
    u.ip = R(1);
    u.mk = 0;
    u.so = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) u.U[c] = u.u[c] = R(0);
    if (!own || !has(q)) return;
    const unsigned k = unsigned(zwrap(q, g.nz)) * nxy + unsigned(n0.off);
#pragma unroll
    for (int c = 0; c < 3; ++c) u.u[c] = a.u[c][k];
    u.mk = a.mask[k];
    if (a.exact) u.ip = a.inv1pa[k];
    if (a.sens_mode) {
      u.dA = a.dA3[k];
      if constexpr (TH) u.dB = a.dB[k];
      if (a.sens_mode == 1) u.so = a.sens[k];
    }
  };
  // the planes z0 - 2 .. z0 in the slots, z0 + 1 in flight
  load(base);
  store(base);
  load(base + 1);
  store(base + 1);
  load(base + 2);
  store(base + 2);
  load(base + 3);
  ColIn<R> c0, c1;
  col_in(n0, t.z0 - 1, c0);
  col_in(n1, t.z0 - 1, c1);
  AdjIn<R> ucur, unext;
  upd_in(INT_MIN, ucur);
  R Mc[14];
#pragma unroll
  for (int i = 0; i < 14; ++i) Mc[i] = R(0);
  R zm1[6], zc[6], zn[6];
  const R z0v[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
#pragma unroll
  for (int f = 0; f < 6; ++f) zm1[f] = zc[f] = R(0);
  // FP32, three barriers per plane: the pulls of plane s read three
  // coefficient slots; after them plane s + 2 takes the slot of plane s - 1
  // and the update of plane s - 1 reads the in-plane moment fields; after
  // that plane s replaces them
  if constexpr (LEAN) {
    for (int s = t.z0 - 1; s <= t.z1; ++s) {
      lds_barrier();
      ColIn<R> c0n, c1n;
      col_in(n0, s + 1 <= t.z1 ? s + 1 : INT_MIN, c0n);
      col_in(n1, s + 1 <= t.z1 ? s + 1 : INT_MIN, c1n);
      upd_in(s >= t.z0 && s < t.z1 ? s : INT_MIN, unext);
      // (in FP64 the own column's reads wait until the ring column is done:
      // held across its pulls they cost more registers than they save)
      R M[14], Mr[14], Mb0[14], u00;
      if constexpr (sizeof(R) == 4) bnd_in(c0, true, Mb0, u00);
      {
        R Mb1[14], u01;
        bnd_in(c1, false, Mb1, u01);
        moments(n1, c1, s, Mb1, u01, Mr);
      }
      if constexpr (sizeof(R) != 4) bnd_in(c0, true, Mb0, u00);
      moments(n0, c0, s, Mb0, u00, M);
      lds_barrier();
      if (s + 2 <= last) store(s + 2);
      if (s + 3 <= last) load(s + 3);
      zn[0] = M[6];
      zn[1] = M[8];
      zn[2] = M[9];
      zn[3] = TH ? M[13] : R(0);
      zn[4] = c0.T;
      zn[5] = c0.B;
      if (own && s - 1 >= t.z0) {
        AdjIn<R> cu = ucur;
        cu.r = Mc[0];
#pragma unroll
        for (int c = 0; c < 3; ++c) cu.U[c] = Mc[1 + c];
        cu.Tt = TH ? Mc[10] : R(0);
        R zd[6];
#pragma unroll
        for (int f = 0; f < 6; ++f) zd[f] = dz3(0, zc[f], zm1[f], zn[f], R(0));
        adj3_update<R, TH>(a, g, unsigned(zwrap(s - 1, g.nz)) * nxy + unsigned(n0.off), L.e[0],
                           n0.ci, n0.ex, n0.ey, 0, cu, zd, zc, zm1, zn, z0v);
      }
      // the z-window moments next to the end planes, for alks3e<ENDS>
      if (!pz && own && c0.valid && !c0.ne && s >= t.z0 && s < t.z1 &&
          (s <= 2 || s >= g.nz - 3)) {
        a.m[6 * N + c0.k] = M[6];
        a.m[8 * N + c0.k] = M[8];
        a.m[9 * N + c0.k] = M[9];
        if constexpr (TH) a.m[13 * N + c0.k] = M[13];
      }
      lds_barrier();
      store_e(n1, Mr, c1, 0);
      store_e(n0, M, c0, 0);
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        zm1[f] = zc[f];
        zc[f] = zn[f];
      }
#pragma unroll
      for (int i = 0; i < 14; ++i) Mc[i] = M[i];
      ucur = unext;
      c0 = c0n;
      c1 = c1n;
    }
  } else {
    // FP64, one barrier per plane: plane s + 2 goes to the fourth slot and
    // the moment fields alternate between two planes
    for (int s = t.z0 - 1; s <= t.z1; ++s) {
      lds_barrier();
      if (s + 2 <= last) store(s + 2);
      if (s + 3 <= last) load(s + 3);
      ColIn<R> c0n, c1n;
      col_in(n0, s + 1 <= t.z1 ? s + 1 : INT_MIN, c0n);
      col_in(n1, s + 1 <= t.z1 ? s + 1 : INT_MIN, c1n);
      upd_in(s >= t.z0 && s < t.z1 ? s : INT_MIN, unext);
      // (in FP64 the own column's reads wait until the ring column is done:
      // held across its pulls they cost more registers than they save)
      R M[14], Mb0[14], u00;
      if constexpr (sizeof(R) == 4) bnd_in(c0, true, Mb0, u00);
      {
        R Mr[14], Mb1[14], u01;
        bnd_in(c1, false, Mb1, u01);
        moments(n1, c1, s, Mb1, u01, Mr);
        store_e(n1, Mr, c1, s & 1);
      }
      if constexpr (sizeof(R) != 4) bnd_in(c0, true, Mb0, u00);
      moments(n0, c0, s, Mb0, u00, M);
      store_e(n0, M, c0, s & 1);
      zn[0] = M[6];
      zn[1] = M[8];
      zn[2] = M[9];
      zn[3] = TH ? M[13] : R(0);
      zn[4] = c0.T;
      zn[5] = c0.B;
      if (own && s - 1 >= t.z0) {
        AdjIn<R> cu = ucur;
        cu.r = Mc[0];
#pragma unroll
        for (int c = 0; c < 3; ++c) cu.U[c] = Mc[1 + c];
        cu.Tt = TH ? Mc[10] : R(0);
        R zd[6];
#pragma unroll
        for (int f = 0; f < 6; ++f) zd[f] = dz3(0, zc[f], zm1[f], zn[f], R(0));
        adj3_update<R, TH>(a, g, unsigned(zwrap(s - 1, g.nz)) * nxy + unsigned(n0.off),
                           L.e[(s - 1) & 1], n0.ci, n0.ex, n0.ey, 0, cu, zd, zc, zm1, zn, z0v);
      }
      // the z-window moments next to the end planes, for alks3e<ENDS>
      if (!pz && own && c0.valid && !c0.ne && s >= t.z0 && s < t.z1 &&
          (s <= 2 || s >= g.nz - 3)) {
        a.m[6 * N + c0.k] = M[6];
        a.m[8 * N + c0.k] = M[8];
        a.m[9 * N + c0.k] = M[9];
        if constexpr (TH) a.m[13 * N + c0.k] = M[13];
      }
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        zm1[f] = zc[f];
        zc[f] = zn[f];
      }
#pragma unroll
      for (int i = 0; i < 14; ++i) Mc[i] = M[i];
      ucur = unext;
      c0 = c0n;
      c1 = c1n;
    }
  }
}

// objective sum over tagged nodes (steady runs): pressure-drop tags of
// drho, or the probe enthalpy flux u_x T. TS blocks stride over the nodes in
// a fixed order and leave one partial sum each.
constexpr int TS = 256;
template <typename R>
__global__ __launch_bounds__(NT3) void tag_sum3_kernel(Geo3 g, const uint8_t* __restrict__ mask,
                                                       const R* d, const R* ux, const R* T,
                                                       int objective, double* part) {
  __shared__ double red[NT3 / 64];
  double s = 0.0;
  for (int k = int(blockIdx.x) * NT3 + int(threadIdx.x); k < g.N; k += TS * NT3) {
    const int m = mask[k];
    if (objective == 1) {
      if (m & TAG_PROBE3) s += double(ux[k]) * double(T[k]);
    } else {
      if (m & TAG_J_INLET3) s += double(d[k]);
      if (m & TAG_J_OUTLET3) s -= double(d[k]);
    }
  }
  s = block_sum3(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

}  // namespace

int blocks3(int N) {
  const int b = (N + NT3 - 1) / NT3;
  return NXCD * ((b + NXCD - 1) / NXCD);
}

int zblocks3(const Geo3& g) { return ztiles(g.nx, ZX) * ztiles(g.ny, ZY) * zchunks(g); }

namespace {
// planes per chunk so that tiles x chunks fills whole rounds of the kernel's
// resident blocks (one round when the grid allows)
template <typename K>
int zplanes(const Geo3& g, K kernel, int nt = ZT) {
  int dev = 0, ncu = 0, bpc = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, kernel, nt, 0) != hipSuccess ||
      ncu <= 0 || bpc <= 0)
    return 16;
  const int tiles = ztiles(g.nx, ZX) * ztiles(g.ny, ZY);
  int nch = (bpc * ncu) / tiles;
  if (nch < 1) nch = 1;
  if (nch > g.nz / 2) nch = g.nz / 2 > 1 ? g.nz / 2 : 1;
  const int zc = g.nz / nch;
  return zc < 2 ? 2 : zc;
}
}  // namespace

void zplan3(Geo3& g, int rsz) {
  if (rsz == 8) {
    g.zc = g.thermal ? zplanes(g, lks3z_kernel<double, true>) : zplanes(g, lks3z_kernel<double, false>);
    g.zca = g.thermal ? zplanes(g, alks3e_kernel<double, true>)
                      : zplanes(g, alks3e_kernel<double, false>);
    g.zcf = g.thermal ? zplanes(g, alks3f_kernel<double, true>)
                      : zplanes(g, alks3f_kernel<double, false>);
  } else {
    g.zc = g.thermal ? zplanes(g, lks3z_kernel<float, true>) : zplanes(g, lks3z_kernel<float, false>);
    g.zca = g.thermal ? zplanes(g, alks3e_kernel<float, true>)
                      : zplanes(g, alks3e_kernel<float, false>);
    g.zcf = g.thermal ? zplanes(g, alks3f_kernel<float, true>)
                      : zplanes(g, alks3f_kernel<float, false>);
  }
}

int copy_nodes3(const Geo3& g, int* out) {
  const int n3[3] = {g.nx, g.ny, g.nz};
  int n = 0;
  for (int l = 0; l < g.nz; ++l)
    for (int j = 0; j < g.ny; ++j)
      for (int i = 0; i < g.nx; ++i) {
        const int c[3] = {i, j, l};
        int ne = 0;
        for (int ax = 0; ax < 3; ++ax)
          if (!((g.periodic >> ax) & 1) && (c[ax] == 0 || c[ax] == n3[ax] - 1)) ++ne;
        if (ne < 2) continue;
        if (out) out[n] = (l * g.ny + j) * g.nx + i;
        ++n;
      }
  return n;
}

int face_nodes3(const Geo3& g, int* out) {
  const int n3[3] = {g.nx, g.ny, g.nz};
  std::vector<int> bucket[7];  // orientations 0..5, then edges and corners
  for (int l = 0; l < g.nz; ++l)
    for (int j = 0; j < g.ny; ++j)
      for (int i = 0; i < g.nx; ++i) {
        const int c[3] = {i, j, l};
        int ne = 0, o = -1;
        for (int ax = 0; ax < 3; ++ax) {
          if ((g.periodic >> ax) & 1) continue;
          if (c[ax] == 0) { ++ne; o = 2 * ax; }
          else if (c[ax] == n3[ax] - 1) { ++ne; o = 2 * ax + 1; }
        }
        if (ne) bucket[ne >= 2 ? 6 : o].push_back((l * g.ny + j) * g.nx + i);
      }
  int n = 0;
  for (const auto& v : bucket)
    for (int k : v) {
      if (out) out[n] = k;
      ++n;
    }
  return n;
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
  const unsigned nb = unsigned(NXCD * ((zblocks3(g) + NXCD - 1) / NXCD));
  const unsigned nc = unsigned((a.ncopy + NT3 - 1) / NT3);
  if (g.thermal) {
    lks3z_kernel<R, true><<<nb, ZT, 0, s>>>(g, a);
    if (a.ncopy)
      copy3_kernel<R, true><<<nc, NT3, 0, s>>>(g, a.copy, a.ncopy, a.s1[0], a.s1[1], a.s1[2],
                                               a.s1[3], a.s1[4]);
  } else {
    lks3z_kernel<R, false><<<nb, ZT, 0, s>>>(g, a);
    if (a.ncopy)
      copy3_kernel<R, false><<<nc, NT3, 0, s>>>(g, a.copy, a.ncopy, a.s1[0], a.s1[1], a.s1[2],
                                                a.s1[3], a.s1[4]);
  }
}

template <typename R, bool TH>
void launch_alks3_fused(const Geo3& g0, const Adj3Args<R>& a, hipStream_t s) {
  Geo3 g = g0;
  g.zc = g0.zcf;
  const unsigned nz = unsigned(NXCD * ((zblocks3(g) + NXCD - 1) / NXCD));
  const unsigned nf = unsigned((a.nface + NT3 - 1) / NT3);
  if (a.nface) alks3_face_kernel<R, TH><<<nf, NT3, 0, s>>>(g, a);
  alks3f_kernel<R, TH><<<nz, ZT, 0, s>>>(g, a);
  if (!(g.periodic & 4)) {
    const int ends = 2 * ztiles(g.nx, ZX) * ztiles(g.ny, ZY);
    alks3e_kernel<R, TH, true><<<unsigned(NXCD * ((ends + NXCD - 1) / NXCD)), ZT, 0, s>>>(g, a);
  }
}

template <typename R>
void launch_alks3_step(const Geo3& g0, const Adj3Args<R>& a, hipStream_t s) {
  if (g0.fused) {
    if (g0.thermal) launch_alks3_fused<R, true>(g0, a, s);
    else launch_alks3_fused<R, false>(g0, a, s);
    return;
  }
  Geo3 g = g0;
  g.zc = g0.zca;
  const unsigned nb = unsigned(blocks3(g.N));
  const unsigned nz = unsigned(NXCD * ((zblocks3(g) + NXCD - 1) / NXCD));
  const unsigned nf = unsigned((a.nface + NT3 - 1) / NT3);
  if (g.thermal) {
    alks3_pull_kernel<R, true><<<nb, NT3, 0, s>>>(g, a);
    if (a.nface) alks3_face_kernel<R, true><<<nf, NT3, 0, s>>>(g, a);
    alks3e_kernel<R, true><<<nz, ZT, 0, s>>>(g, a);
  } else {
    alks3_pull_kernel<R, false><<<nb, NT3, 0, s>>>(g, a);
    if (a.nface) alks3_face_kernel<R, false><<<nf, NT3, 0, s>>>(g, a);
    alks3e_kernel<R, false><<<nz, ZT, 0, s>>>(g, a);
  }
}

template <typename R>
void launch_tag_sum3(const Geo3& g, const uint8_t* mask, const R* d, const R* ux, const R* T,
                     int objective, double* part, double* out, hipStream_t s) {
  tag_sum3_kernel<R><<<TS, NT3, 0, s>>>(g, mask, d, ux, T, objective, part);
  launch_sum(part, TS, out, s);
}

int tag_sum3_parts() { return TS; }

#define LKS3_INSTANTIATE(R)                                                                   \
  template void launch_coef3<R>(const Geo3&, const uint8_t*, const double*, double, double,  \
                                double, double, double, R*, R*, R*, R*, hipStream_t);        \
  template void launch_init3<R>(const Geo3&, const uint8_t*, const R* const[3], const R*,    \
                                double, R* const[5], hipStream_t);                           \
  template void launch_lks3_step<R>(const Geo3&, const Fwd3Args<R>&, hipStream_t);           \
  template void launch_alks3_step<R>(const Geo3&, const Adj3Args<R>&, hipStream_t);          \
  template void launch_tag_sum3<R>(const Geo3&, const uint8_t*, const R*, const R*, const R*, \
                                   int, double*, double*, hipStream_t);
LKS3_INSTANTIATE(float)
LKS3_INSTANTIATE(double)

}  // namespace lks
