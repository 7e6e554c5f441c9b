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
#include <type_traits>

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

// heat source (eq:heatsource, eq:betagamma): beta = bmax q (1 - g) / (q + g)
// and beta' at design nodes, 0 on the ring
template <typename R>
__global__ void source_coef_kernel(Geo g, const double* __restrict__ gamma, double bmax,
                                   double qb, R* __restrict__ beta, R* __restrict__ dbeta) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.N) return;
  int i = k % g.nx, j = k / g.nx;
  bool ring = !g.periodic && (i == 0 || j == 0 || i == g.nx - 1 || j == g.ny - 1);
  if (ring) {
    beta[k] = R(0);
    dbeta[k] = R(0);
    return;
  }
  double ga = gamma[k];
  beta[k] = R(bmax * qb * (1.0 - ga) / (qb + ga));
  dbeta[k] = R(-bmax * qb * (1.0 + qb) / ((qb + ga) * (qb + ga)));
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

// element e of a small per-thread array by selects, so the array stays in
// registers where the compiler cannot resolve e (a runtime index moves it to
// per-lane scratch memory)
template <typename T, int N>
__device__ inline T pick(const T (&a)[N], int e) {
  T v = a[0];
#pragma unroll
  for (int i = 1; i < N; ++i) v = e == i ? a[i] : v;
  return v;
}

// ---------------------------------------------------------------------------
// block reduction helper (deterministic)
// ---------------------------------------------------------------------------
template <int NT = NTHREADS>
__device__ inline double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < NT / 64; ++w) s += red[w];
  return s;
}

// threads of a one-step block: 512 (8 waves, each stage then walks its
// region in one or two passes) for FP32 tiles of 16 rows and thermal FP32
// tiles of 8 rows; 256 otherwise (measured: the non-thermal 64 x 8 step on
// large grids keeps more tiles in flight with 256)
template <typename R, bool TH, int TY>
constexpr int NT1 =
    (TY == 16 || TY == 4 || (TY == 8 && (TH || sizeof(R) == 8))) ? 512 : NTHREADS;

// ---------------------------------------------------------------------------
// tiles
// ---------------------------------------------------------------------------
// A block owns a tile of TX x TY nodes (the last tile along an axis may be
// up to one node larger or smaller). LDS holds the tile with a 2-node halo
// (raw state, pitch W2) or a 1-node halo (post-collision values, pitch W1).
// Full tiles -- TX x TY, the common case -- walk their rectangles with
// compile-time extents; the others use the runtime extents.
template <int TY>
struct Tile {
  static constexpr int W2 = TX + 1 + 4, H2 = TY + 1 + 4;
  static constexpr int W1 = TX + 1 + 2, H1 = TY + 1 + 2;
};

// Global tile of this block under the XCD-aware mapping, or -1.
__device__ inline int xcd_tile(int T) {
  const int nper = (T + NXCD - 1) / NXCD;
  const int b = blockIdx.x;
  const int tile = (b % NXCD) * nper + b / NXCD;
  return tile < T ? tile : -1;
}

__device__ inline void tile_box(const Geo& g, int tile, int* x0, int* x1, int* y0, int* y1) {
  const int bx = tile % g.ntx, by = tile / g.ntx;
  *x0 = bx * TX;
  *x1 = (bx == g.ntx - 1) ? g.nx : *x0 + TX;
  *y0 = by * g.ty;
  *y1 = (by == g.nty - 1) ? g.ny : *y0 + g.ty;
}

__device__ inline bool block_tile(const Geo& g, int* x0, int* x1, int* y0, int* y1, int* t) {
  const int tile = xcd_tile(g.ntx * g.nty);
  if (tile < 0) return false;
  tile_box(g, tile, x0, x1, y0, y1);
  *t = tile;
  return true;
}

// A tile whose 2-node halo stays inside the domain and whose 1-node halo
// holds no boundary-ring node: no wrap, no ring rule, central differences.
__device__ inline bool interior_tile(const Geo& g, int x0, int x1, int y0, int y1) {
  return x0 >= 2 && y0 >= 2 && x1 <= g.nx - 2 && y1 <= g.ny - 2;
}

// How a tile treats its nodes:
//   K_GEN   every node takes the general rule (wrap-around, bounds, ring
//           rules, one-sided differences): periodic boxes and odd tiles;
//   K_INT   the tile and its halo lie off the ring: every node is interior;
//   K_EDGE  a tile of a bounded domain that meets the ring: the nodes off
//           the ring take the interior rule in the flat walk of the tile,
//           the few ring nodes are gathered into a second walk of their own,
//           so a wave does not pay for the ring rules of one of its lanes.
// The per-node arithmetic is the same function in all three, so the kinds
// give the same bits.
constexpr int K_GEN = 0, K_INT = 1, K_EDGE = 2;

template <bool B>
using BoolC = std::integral_constant<bool, B>;

// true on the boundary ring of a bounded domain, and outside it
__device__ inline bool on_ring(const Geo& g, int i, int j) {
  return i <= 0 || j <= 0 || i >= g.nx - 1 || j >= g.ny - 1;
}

// The ring nodes of the node rectangle [x0, x0 + w) x [y0, y0 + h) clipped
// to a bounded domain: its parts of the columns i = 0 and i = nx - 1, then
// of the rows j = 0 and j = ny - 1 without the end nodes of those rows.
struct RingSet {
  int ry0, bx0, nl, nr, nb;
};

__device__ inline int ring_set(const Geo& g, int x0, int y0, int w, int h, RingSet& s) {
  const int rx0 = max(x0, 0), rx1 = min(x0 + w, g.nx) - 1;
  const int ry0 = max(y0, 0), ry1 = min(y0 + h, g.ny) - 1;
  const int hc = ry1 - ry0 + 1;
  s.ry0 = ry0;
  s.nl = rx0 == 0 ? hc : 0;
  s.nr = rx1 == g.nx - 1 ? hc : 0;
  s.bx0 = max(rx0, 1);
  const int wr = max(min(rx1, g.nx - 2) - s.bx0 + 1, 0);
  s.nb = ry0 == 0 ? wr : 0;
  const int nt = ry1 == g.ny - 1 ? wr : 0;
  return s.nl + s.nr + s.nb + nt;
}

__device__ inline void ring_at(const Geo& g, const RingSet& s, int t, int* i, int* j) {
  if (t < s.nl) {
    *i = 0;
    *j = s.ry0 + t;
  } else if (t < s.nl + s.nr) {
    *i = g.nx - 1;
    *j = s.ry0 + t - s.nl;
  } else if (t < s.nl + s.nr + s.nb) {
    *i = s.bx0 + t - s.nl - s.nr;
    *j = 0;
  } else {
    *i = s.bx0 + t - s.nl - s.nr - s.nb;
    *j = g.ny - 1;
  }
}

// Visit the ring nodes (i, j) of a rectangle, one per thread from the last
// thread of the block down (the flat walks leave those idle most often).
template <int NT = NTHREADS, typename F>
__device__ inline void ring_loop(const Geo& g, int x0, int y0, int w, int h, F&& f) {
  RingSet s;
  const int n = ring_set(g, x0, y0, w, h, s);
  for (int t = NT - 1 - int(threadIdx.x); t < n; t += NT) {
    int i, j;
    ring_at(g, s, t, &i, &j);
    f(i, j);
  }
}

// Visit the positions (lx, ly) of a w x h rectangle, NT threads, flat order.
template <bool FULL, int WC, int HC, int NT = NTHREADS, typename F>
__device__ inline void rect_loop(int w, int h, F&& f) {
  if constexpr (FULL) {
    constexpr int n = WC * HC;
#pragma unroll
    for (int p0 = 0; p0 < n; p0 += NT) {
      const int p = p0 + int(threadIdx.x);
      if (p < n) f(p % WC, p / WC);
    }
  } else {
    const int n = w * h;
    for (int p = threadIdx.x; p < n; p += NT) f(p % w, p / w);
  }
}

// Walk the region of a tile grown by h nodes on every side (w x hh
// positions; compile-time extents WC x HC for full tiles): fn(rule, lx, ly,
// i, j) at each node of the region in the domain, where (lx, ly) is the
// region position and rule is BoolC<true> for the interior rule. K_GEN
// wraps a periodic box and skips positions outside a bounded one; K_EDGE
// walks the nodes off the ring first and its ring nodes after.
template <int KIND, bool FULL, int WC, int HC, int NT = NTHREADS, typename F>
__device__ inline void region_walk(const Geo& g, int x0, int y0, int h, int w, int hh, F&& fn) {
  rect_loop<FULL, WC, HC, NT>(w, hh, [&](int lx, int ly) {
    int i = x0 + lx - h, j = y0 + ly - h;
    if constexpr (KIND == K_EDGE) {
      if (on_ring(g, i, j)) return;
    } else if constexpr (KIND == K_GEN) {
      if (g.periodic) {
        i = wrapi(i, g.nx);
        j = wrapi(j, g.ny);
      } else if (i < 0 || j < 0 || i >= g.nx || j >= g.ny) {
        return;
      }
    }
    fn(BoolC<KIND != K_GEN>(), lx, ly, i, j);
  });
  if constexpr (KIND == K_EDGE)
    ring_loop<NT>(g, x0 - h, y0 - h, w, hh,
                  [&](int i, int j) { fn(BoolC<false>(), i - x0 + h, j - y0 + h, i, j); });
}

// interior_tile for the two-step kernels, whose tiles carry a 4-node halo
__device__ inline bool interior_tile2(const Geo& g, int x0, int x1, int y0, int y1) {
  return x0 >= 4 && y0 >= 4 && x1 <= g.nx - 4 && y1 <= g.ny - 4;
}

// Load NF fields of the tile plus an H-node halo into LDS arrays of pitch P
// (zeros outside a non-periodic domain). For full tiles (TX x TY) every load
// is issued before any is used so that their latencies overlap.
template <typename R, bool FULL, int TY, int H, int P, int NF, bool INT = false,
          int NT = NTHREADS>
__device__ inline void load_halo(const Geo& g, int x0, int y0, int tw, int th,
                                 const R* const (&src)[NF], R* const (&dst)[NF]) {
  auto node = [&](int lx, int ly, int* k) {
    int i = x0 + lx - H, j = y0 + ly - H;
    bool in = true;
    if constexpr (INT) {
      *k = j * g.nx + i;
      return true;
    }
    if (g.periodic) {
      i = wrapi(i, g.nx);
      j = wrapi(j, g.ny);
    } else {
      in = i >= 0 && i < g.nx && j >= 0 && j < g.ny;
    }
    *k = in ? j * g.nx + i : 0;
    return in;
  };
  if constexpr (FULL) {
    constexpr int WC = TX + 2 * H, HC = TY + 2 * H, n = WC * HC;
    constexpr int NP = (n + NT - 1) / NT;
    int kk[NP], pp[NP];
    bool ok[NP];
#pragma unroll
    for (int e = 0; e < NP; ++e) {
      const int p = e * NT + int(threadIdx.x);
      const int lx = p % WC, ly = p / WC;
      ok[e] = node(lx, ly, &kk[e]) && p < n;
      if (p >= n) kk[e] = 0;
      pp[e] = p < n ? ly * P + lx : -1;
    }
    R v[NF][NP];
#pragma unroll
    for (int e = 0; e < NP; ++e)
#pragma unroll
      for (int f = 0; f < NF; ++f) v[f][e] = src[f][kk[e]];
#pragma unroll
    for (int e = 0; e < NP; ++e)
      if (pp[e] >= 0)
#pragma unroll
        for (int f = 0; f < NF; ++f) dst[f][pp[e]] = ok[e] ? v[f][e] : R(0);
  } else {
    rect_loop<false, 1, 1, NT>(tw + 2 * H, th + 2 * H, [&](int lx, int ly) {
      int k;
      const bool in = node(lx, ly, &k);
      const int p = ly * P + lx;
#pragma unroll
      for (int f = 0; f < NF; ++f) dst[f][p] = in ? src[f][k] : R(0);
    });
  }
}

// LDS finite difference along x or y at position p of a field with the
// given row step, for node coordinate c along that axis (second-order
// central, one-sided at the two ends of a non-periodic axis).
template <typename R>
__device__ inline R lds_d(const R* s, int p, int step, int c, int n, int periodic) {
  if (periodic || (c > 0 && c < n - 1)) return R(0.5) * (s[p + step] - s[p - step]);
  if (c == 0) return R(0.5) * (R(-3) * s[p] + R(4) * s[p + step] - s[p + 2 * step]);
  return R(0.5) * (R(3) * s[p] - R(4) * s[p - step] + s[p - 2 * step]);
}

// lds_d for a position whose tile is interior (INT: the tile and a 2-node
// halo lie off the boundary ring and need no wrap), where the central
// difference always applies
template <bool INT, typename R>
__device__ inline R lds_dx(const R* s, int p, int step, int c, int n, int periodic) {
  if constexpr (INT) return R(0.5) * (s[p + step] - s[p - step]);
  else return lds_d(s, p, step, c, n, periodic);
}

// the same difference of the product a*b of two LDS fields with their own
// positions and row steps
template <bool INT, typename R>
__device__ inline R lds_dxp(const R* a, int pa, int sa, const R* b, int pb, int sb, int c, int n,
                            int periodic) {
  auto at = [&](int o) { return a[pa + o * sa] * b[pb + o * sb]; };
  if (INT || periodic || (c > 0 && c < n - 1)) return R(0.5) * (at(1) - at(-1));
  if (c == 0) return R(0.5) * (R(-3) * at(0) + R(4) * at(1) - at(2));
  return R(0.5) * (R(3) * at(0) - R(4) * at(-1) + at(-2));
}

// ---------------------------------------------------------------------------
// LKS step
// ---------------------------------------------------------------------------
// One LKS step, level n -> n+1 (eq:rho, eq:u, eq:T with eq:feq2 and eq:geq2
// read as g_i^eq = w_i [T (1 + 3 c.u) + B c.grad T], and the implicit
// Brinkman term of eq:lbef_ex giving u = U* / (1 + alpha)).
// Density is carried as drho = rho - 1: the constant part of f_i^eq adds 1
// to the density and 0 to the momentum, so LDS holds f'_i = f_i^eq - w_i.
//   stage A0  the raw state of the tile and a 2-node halo into LDS;
//   stage A1  the nine post-collision values f'_i (and g_i) of every node of
//             the tile and a 1-node halo, gradients from LDS;
//   stage B   every tile node pulls f'_i(x - c_i) from LDS. Boundary nodes
//             complete the density (velocity node), normal velocity
//             (pressure node) or temperature (adiabatic node) from the moment
//             balance of the pulled populations; corners copy density and
//             temperature from their y-neighbour, whose thread writes them.
template <typename R, bool TH, int TY>
struct FwdLds {
  using TL = Tile<TY>;
  R d[TL::W2 * TL::H2], u[TL::W2 * TL::H2], v[TL::W2 * TL::H2];
  R T[TH ? TL::W2 * TL::H2 : 1], B[TH ? TL::W2 * TL::H2 : 1];
  R f[9][TL::W1 * TL::H1];
  // thermal: W = 3 T u + B grad T of each node (x, y); its nine g_i follow
  // from T and W, so the puller forms them
  R gq[TH ? 2 : 1][TH ? TL::W1 * TL::H1 : 1];
  double red[8];  // one per wave, up to 512 threads
};

// Stage A1 at one node (i, j): the post-collision values f'_i (and g_i)
// from the raw fields in LDS (pitch PR, position pr), stored at position pf
// of the post-collision arrays f and gq (each direction SF values apart).
template <typename R, bool TH, int PR, int SF, bool INT = false>
__device__ inline void fwd_collide(const Geo& g, R A, const R* ld, const R* lu, const R* lv,
                                   const R* lT, const R* lB, int pr, int i, int j, R* f, R* gq,
                                   int pf) {
#pragma clang fp contract(on)
  const R d = ld[pr], ux = lu[pr], uy = lv[pr];
  const R uxx = lds_dx<INT>(lu, pr, 1, i, g.nx, g.periodic);
  const R uxy = lds_dx<INT>(lu, pr, PR, j, g.ny, g.periodic);
  const R uyx = lds_dx<INT>(lv, pr, 1, i, g.nx, g.periodic);
  const R uyy = lds_dx<INT>(lv, pr, PR, j, g.ny, g.periodic);
  // f'_i = w_i [P + 3 c.u + cx^2 Xx + cy^2 Yy + cx cy Xy]
  const R P = d - R(1.5) * (ux * ux + uy * uy);
  const R Xx = R(4.5) * ux * ux + R(2) * A * uxx;
  const R Yy = R(4.5) * uy * uy + R(2) * A * uyy;
  const R Xy = R(9) * ux * uy + R(2) * A * (uxy + uyx);
  const R u3x = R(3) * ux, u3y = R(3) * uy;
  const R w0 = R(4.0 / 9), w1 = R(1.0 / 9), w5 = R(1.0 / 36);
  const R diag = P + Xx + Yy;
  f[0 * SF + pf] = w0 * P;
  f[1 * SF + pf] = w1 * (P + u3x + Xx);
  f[2 * SF + pf] = w1 * (P + u3y + Yy);
  f[3 * SF + pf] = w1 * (P - u3x + Xx);
  f[4 * SF + pf] = w1 * (P - u3y + Yy);
  f[5 * SF + pf] = w5 * (diag + u3x + u3y + Xy);
  f[6 * SF + pf] = w5 * (diag - u3x + u3y - Xy);
  f[7 * SF + pf] = w5 * (diag - u3x - u3y + Xy);
  f[8 * SF + pf] = w5 * (diag + u3x - u3y - Xy);
  if constexpr (TH) {
    const R T = lT[pr];
    const R Bk = lB[pr];
    const R Wx = R(3) * T * ux + Bk * lds_dx<INT>(lT, pr, 1, i, g.nx, g.periodic);
    const R Wy = R(3) * T * uy + Bk * lds_dx<INT>(lT, pr, PR, j, g.ny, g.periodic);
    gq[0 * SF + pf] = Wx;
    gq[1 * SF + pf] = Wy;
  }
}

// g_q = w_q [T + c_q.W] (eq:geq2) of the node whose temperature is T and
// whose W is (Wx, Wy)
template <typename R>
__device__ inline R g_eq(int q, R T, R Wx, R Wy) {
#pragma clang fp contract(on)
  const R w0 = R(4.0 / 9), w1 = R(1.0 / 9), w5 = R(1.0 / 36);
  switch (q) {
    case 0: return w0 * T;
    case 1: return w1 * (T + Wx);
    case 2: return w1 * (T + Wy);
    case 3: return w1 * (T - Wx);
    case 4: return w1 * (T - Wy);
    case 5: return w5 * (T + Wx + Wy);
    case 6: return w5 * (T - Wx + Wy);
    case 7: return w5 * (T - Wx - Wy);
    default: return w5 * (T + Wx - Wy);
  }
}

// Stage B at one node (i, j), not a corner: pull f'_i(x - c_i) from the
// post-collision arrays (pitch PF, position pf) and form the new state;
// ring nodes complete it from the moment balance. `level` is the new level
// (inflow factor of velocity nodes).
template <typename R, bool TH, int PF, int SF, int PR, bool INT = false>
__device__ inline void fwd_pull(const Geo& g, const FwdArgs<R>& a, const R* lf, const R* lg,
                                const R* lT, int pf, int pr, int i, int j, int k, int m, R s,
                                int level, R& dn, R& uxn, R& uyn, R& Tn) {
#pragma clang fp contract(on)
  const int fc = (INT || g.periodic) ? FLOW_INTERIOR : (m & 3);
  R f[9], gg[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) f[q] = lf[q * SF + pf - CX[q] - CY[q] * PF];
  if constexpr (TH) {
    // g_q(x - c_q) from the source's T (raw fields, pitch PR, position pr
    // of this node) and W (pitch PF)
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const int pw = pf - CX[q] - CY[q] * PF;
      gg[q] = g_eq<R>(q, lT[pr - CX[q] - CY[q] * PR], lg[pw], lg[SF + pw]);
    }
  }
  Tn = R(0);
  if (fc == FLOW_INTERIOR) {
    dn = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
    R Ux = f[1] - f[3] + f[5] - f[6] - f[7] + f[8];
    R Uy = f[2] - f[4] + f[5] + f[6] - f[7] - f[8];
    if constexpr (TH) {
      Tn = gg[0] + gg[1] + gg[2] + gg[3] + gg[4] + gg[5] + gg[6] + gg[7] + gg[8];
      // heat source Q = beta (1 - T) at the new level (eq:lbeg_ex,
      // eq:heatsource): T (1 + beta) = T* + beta
      if (a.beta) {
        const R b = a.beta[k];
        Tn = (Tn + b) / (R(1) + b);
      }
      // Boussinesq force at the new level, u (1 + alpha) = U* + G
      // (eq:lbef_ex, eq:boussinesqforce); zero when g beta is zero
      const R dT = Tn - R(g.Tref);
      Ux += R(g.gbx) * dT;
      Uy += R(g.gby) * dT;
    }
    uxn = Ux * s;
    uyn = Uy * s;
    return;
  }
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
    const double fac = a.ufac[level];
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
    // heat-flux node: -q.n = qbar with q = sum c_i g_i - u T (Sec. 2.4); Tb
    // holds qbar there (0: adiabatic)
    if (((m >> 2) & 3) == THERM_DIRICHLET) Tn = a.Tb[k];
    else Tn = (S0g + R(2) * Spg + a.Tb[k]) / (R(1) + un);
  }
}

// corners take density and temperature from their y-neighbour at the new
// level: the neighbour (i, 1) or (i, ny-2) of a corner column hands its
// values to `put` for the corner row
template <typename Put>
__device__ inline void corner_from(const Geo& g, int i, int j, Put&& put) {
  if (g.periodic || (i != 0 && i != g.nx - 1)) return;
  if (j == 1) put(0);
  if (j == g.ny - 2) put(g.ny - 1);
}

// the objective's term of node k with class m at a new level (pressure drop,
// probe enthalpy flux, heat exchange or heated-node temperature)
template <typename R, bool TH>
__device__ inline void obj_add(const FwdArgs<R>& a, int m, int k, R dn, R uxn, R Tn,
                               double& part) {
  if (a.objective == 1) {
    if (m & TAG_PROBE) part += double(uxn) * double(Tn);
  } else if (a.objective == 2) {
    if constexpr (TH) part += double(a.beta[k]) * (double(Tn) - 1.0);
  } else if (a.objective == 3) {
    if (m & TAG_PROBE) part += double(Tn);
  } else {
    if (m & TAG_J_INLET) part += double(dn);
    if (m & TAG_J_OUTLET) part -= double(dn);
  }
}

template <typename R, bool TH, int TY, bool FULL, int KIND, int NT = NT1<R, TH, TY>>
__device__ void lks_tile(const Geo& g, const FwdArgs<R>& a, FwdLds<R, TH, TY>& L, int x0, int y0,
                         int tw, int th, int tile) {
  using TL = Tile<TY>;
  constexpr int W2 = TL::W2, W1 = TL::W1, SF = TL::W1 * TL::H1;
  constexpr bool INT = KIND == K_INT, EDGE = KIND == K_EDGE;
  const R A = R(g.A);
  if constexpr (FULL) {
    tw = TX;
    th = TY;
  }
  // node-local inputs of stage B, loaded before the first barrier (full tiles)
  constexpr int NB = FULL ? (TX * TY + NT - 1) / NT : 1;
  int mpre[NB];
  R spre[NB];
  if constexpr (FULL) {
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int p = e * NT + int(threadIdx.x);
      if (p >= TX * TY) break;  // more threads than tile nodes
      const int k = (y0 + p / TX) * g.nx + x0 + p % TX;
      mpre[e] = a.mask[k];
      spre[e] = a.inv1pa[k];
    }
  }

  if constexpr (TH) {
    const R* src[5] = {a.d0, a.ux0, a.uy0, a.T0, a.B};
    R* dst[5] = {L.d, L.u, L.v, L.T, L.B};
    load_halo<R, FULL, TY, 2, W2, 5, INT, NT>(g, x0, y0, tw, th, src, dst);
  } else {
    const R* src[3] = {a.d0, a.ux0, a.uy0};
    R* dst[3] = {L.d, L.u, L.v};
    load_halo<R, FULL, TY, 2, W2, 3, INT, NT>(g, x0, y0, tw, th, src, dst);
  }
  __syncthreads();

  region_walk<KIND, FULL, TX + 2, TY + 2, NT>(g, x0, y0, 1, tw + 2, th + 2,
                                          [&](auto in, int lx, int ly, int i, int j) {
    fwd_collide<R, TH, W2, SF, decltype(in)::value>(g, A, L.d, L.u, L.v, L.T, L.B,
                                                    (ly + 1) * W2 + lx + 1, i, j, &L.f[0][0],
                                                    &L.gq[0][0], ly * W1 + lx);
  });
  __syncthreads();

  double part = 0.0;
  // the pull, new state and objective term of node (i, j) with mask m
  auto pull = [&](auto in, int lx, int ly, int i, int j, int m, R s) {
    constexpr bool I = decltype(in)::value;
    const int k = j * g.nx + i;
    if (!I && !g.periodic && (m & 3) == FLOW_CORNER) return;
    R dn, uxn, uyn, Tn;
    fwd_pull<R, TH, W1, SF, W2, I>(g, a, &L.f[0][0], &L.gq[0][0], L.T, (ly + 1) * W1 + lx + 1,
                                   (ly + 2) * W2 + lx + 2, i, j, k, m, s, a.level_out, dn, uxn,
                                   uyn, Tn);
    if constexpr (!I)
      corner_from(g, i, j, [&](int jc) {
        const int kc = jc * g.nx + i;
        a.d1[kc] = dn;
        a.ux1[kc] = R(0);
        a.uy1[kc] = R(0);
        if constexpr (TH) a.T1[kc] = Tn;
      });
    a.d1[k] = dn;
    a.ux1[k] = uxn;
    a.uy1[k] = uyn;
    if constexpr (TH) a.T1[k] = Tn;
    if (a.acc) obj_add<R, TH>(a, m, k, dn, uxn, Tn, part);
  };
  int e = 0;
  rect_loop<FULL, TX, TY, NT>(tw, th, [&](int lx, int ly) {
    const int i = x0 + lx, j = y0 + ly;
    int m;
    R s;
    if constexpr (FULL) {
      m = mpre[e];
      s = spre[e];
      ++e;
      if constexpr (EDGE)
        if (on_ring(g, i, j)) return;
    } else {
      if constexpr (EDGE)
        if (on_ring(g, i, j)) return;
      const int k = j * g.nx + i;
      m = a.mask[k];
      s = a.inv1pa[k];
    }
    pull(BoolC<INT || EDGE>(), lx, ly, i, j, m, s);
  });
  if constexpr (EDGE)
    ring_loop<NT>(g, x0, y0, tw, th, [&](int i, int j) {
      const int k = j * g.nx + i;
      pull(BoolC<false>(), i - x0, j - y0, i, j, int(a.mask[k]), a.inv1pa[k]);
    });
  if (a.acc) {
    double s = block_sum<NT>(part, L.red);
    if (threadIdx.x == 0) a.acc[tile] += s;
  }
}

template <typename R, bool TH, int TY>
__global__ __launch_bounds__((NT1<R, TH, TY>)) void lks_step_kernel(Geo g, FwdArgs<R> a) {
  __shared__ FwdLds<R, TH, TY> L;
  int x0, x1, y0, y1, tile;
  if (!block_tile(g, &x0, &x1, &y0, &y1, &tile)) return;
  const int tw = x1 - x0, th = y1 - y0;
  if (tw != TX || th != TY) {
    if (g.periodic) lks_tile<R, TH, TY, false, K_GEN>(g, a, L, x0, y0, tw, th, tile);
    else lks_tile<R, TH, TY, false, K_EDGE>(g, a, L, x0, y0, tw, th, tile);
  } else if (interior_tile(g, x0, x1, y0, y1)) {
    lks_tile<R, TH, TY, true, K_INT>(g, a, L, x0, y0, tw, th, tile);
  } else if (g.periodic) {
    lks_tile<R, TH, TY, false, K_GEN>(g, a, L, x0, y0, tw, th, tile);
  } else {
    lks_tile<R, TH, TY, true, K_EDGE>(g, a, L, x0, y0, tw, th, tile);
  }
}

// ---------------------------------------------------------------------------
// ALKS step
// ---------------------------------------------------------------------------
// the completion of ring_moments with the operator op of orientation o and
// flow type v (0 velocity, 1 pressure node)
template <typename R, bool TH, typename OP>
__device__ inline void ring_apply(OP op, int v, int o, const AdjArgs<R>& a, const R* sTn, int p2,
                                  int k, int m, const R f[9], const R gq[9], R mom[9]) {
  R kappa = R(0), gu[3] = {R(0), R(0), R(0)};
  const int nx_ = o == 0 ? -1 : (o == 1 ? 1 : 0);
  const int ny_ = o == 2 ? -1 : (o == 3 ? 1 : 0);
  if constexpr (TH) {
    if (((m >> 2) & 3) == THERM_DIRICHLET) {
#pragma nounroll
      for (int c = 0; c < 3; ++c) {
        R t = R(0);
#pragma unroll
        for (int q = 0; q < 9; ++q) t += op->Ld[c][q] * gq[q];
        gu[c] = t;
      }
    } else {
      const R un = a.ux[k] * R(nx_) + a.uy[k] * R(ny_);
      // zero-flux completion in Schur form (no row seed)
      R num = R(0);
#pragma unroll
      for (int q = 0; q < 9; ++q) num += (op->ga[q] - un * op->ge[q]) * gq[q];
      const R den = op->A0 - R(2) * un * op->A1 + un * un * op->A2;
      kappa = -num / den;
#pragma nounroll
      for (int c = 0; c < 3; ++c) {
        R t = R(0);
#pragma unroll
        for (int q = 0; q < 9; ++q) t += op->Lg0[c][q] * gq[q];
        gu[c] = t - kappa * (op->hc[c] - un * op->h1[c]);
      }
    }
  }
  // boundary seed of the pressure-drop objective: its derivative with
  // respect to the boundary pressure, the same in every row
  R s = R(0);
  if (m & TAG_J_INLET) s += R(a.seed_dp);
  if (m & TAG_J_OUTLET) s -= R(a.seed_dp);
  const R kT = TH ? kappa * sTn[p2] : R(0);
  R fu[3];
#pragma nounroll
  for (int c = 0; c < 3; ++c) {
    R t = op->Ls[v][c] * s + op->Lk[v][c] * kT;
#pragma unroll
    for (int q = 0; q < 9; ++q) t += op->Lf[v][c][q] * f[q];
    fu[c] = t;
  }
  R r = R(0), Ux = R(0), Uy = R(0), sxx = R(0), sxy = R(0), syy = R(0);
  R Tt = R(0), qx = R(0), qy = R(0);
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const R wf = R(WD[q]) * f[q];
    r += wf;
    if (CX[q]) Ux += R(CX[q]) * wf;
    if (CY[q]) Uy += R(CY[q]) * wf;
    if (CX[q]) sxx += wf;
    if (CX[q] * CY[q]) sxy += R(CX[q] * CY[q]) * wf;
    if (CY[q]) syy += wf;
    if constexpr (TH) {
      const R wg = R(WD[q]) * gq[q];
      Tt += wg;
      if (CX[q]) qx += R(CX[q]) * wg;
      if (CY[q]) qy += R(CY[q]) * wg;
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const R cx = op->ucx[c], cy = op->ucy[c];
    const R wf = op->uw[c] * fu[c];
    r += wf;
    Ux += cx * wf;
    Uy += cy * wf;
    sxx += cx * cx * wf;
    sxy += cx * cy * wf;
    syy += cy * cy * wf;
    if constexpr (TH) {
      const R wg = op->uw[c] * gu[c];
      Tt += wg;
      qx += cx * wg;
      qy += cy * wg;
    }
  }
  if constexpr (TH) {
    // heat-sink objective: the heated node's temperature is the flux closure
    // T (1 + u.n) = S0 + 2 S+ + qbar of the arriving populations, so
    // seed_bt w^cl / (1 + u.n) (w^cl = 1 along the wall, 2 moving outwards,
    // 0 inwards) leaves every completed adjoint population; its weighted
    // moments are -seed/(1 + u.n) on T~ and -seed/(1 + u.n) n/3 on q~
    if ((m & TAG_PROBE) && a.seed_bt != 0.0) {
      const R sb = R(a.seed_bt) / (R(1) + a.ux[k] * R(nx_) + a.uy[k] * R(ny_));
      Tt -= sb;
      qx -= sb * R(nx_) / R(3);
      qy -= sb * R(ny_) / R(3);
    }
    // exact mode: the temperature of a prescribed-temperature node does not
    // depend on the populations that arrive there, so their adjoint is zero
    if (a.exact && ((m >> 2) & 3) == THERM_DIRICHLET) Tt = qx = qy = R(0);
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

// Least-squares completion of the adjoint populations at a ring node (see
// RingOp): the known populations f~_i = rho~ + c_i.V and g~_i = Theta at
// x + c_i come from LDS (the unknown directions point outside the domain,
// where LDS holds zeros); returns the raw moments rho~, U~, s~ (xx, xy, yy),
// T~, q~ of the completed set.
template <typename R, bool TH, int W2>
__device__ void ring_moments(const Geo& g, const AdjArgs<R>& a, const R* sr, const R* svx,
                             const R* svy, const R* sth, const R* sTn, int p2, int i, int j,
                             int k, int m, R mom[9]) {
  const int o = (i == 0) ? 0 : (i == g.nx - 1 ? 1 : (j == 0 ? 2 : 3));
  const int v = (m & 3) == FLOW_VELOCITY ? 0 : 1;
  R f[9], gq[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const int p = p2 + CX[q] + CY[q] * W2;
    R e = sr[p];
    if (CX[q] > 0) e += svx[p];
    if (CX[q] < 0) e -= svx[p];
    if (CY[q] > 0) e += svy[p];
    if (CY[q] < 0) e -= svy[p];
    f[q] = e;
    if constexpr (TH) gq[q] = sth[p];
  }
  // a wave whose lanes share orientation and node type reads the operator
  // through the scalar unit; mixed waves read it per lane
  const int key = 2 * o + v;
  const int uk = __builtin_amdgcn_readfirstlane(key);
  if (__all(key == uk))
    ring_apply<R, TH>(as_scalar(a.ops) + (uk >> 1), uk & 1, uk >> 1, a, sTn, p2, k, m, f, gq,
                      mom);
  else
    ring_apply<R, TH>(a.ops + o, v, o, a, sTn, p2, k, m, f, gq, mom);
}

// One ALKS step, adjoint level n+1 -> n. The adjoint state is kept as the
// coefficients of the adjoint equilibria, f~_i^eq = rho~ + c_i.V (eq:afeq)
// and g~_i^eq = Theta (eq:ageq), so a step needs the forward state of one
// level only:
//   stage A0  the level-n+1 coefficients of the tile and a 2-node halo (and
//             T^n, B for the thermal terms) into LDS;
//   stage A1  weighted pull of the equilibria from the 8 neighbours
//             (eq:ap..eq:aq), or the least-squares completion on ring
//             nodes, for the tile and a 1-node halo; corners copy their
//             y-neighbour;
//   stage B   the local terms of eq:albef_ex / eq:albeg_ex at level n
//             (seeds, 3 T q~ coupling, implicit Brinkman
//             u~ = (U~ + T q~ - seed) / (1 + alpha)), then
//             V = 3 u~ + 9 s~ u - 3 rho~ u - 2A div s~ and
//             Theta = T~ + 3 q~.u - B div q~ - grad B . q~ with the
//             level-n state, and the sensitivity
//             3 alpha' u.u~ - B' grad T . q~ (Sec. 2.5).
template <typename R, bool TH, int TY>
struct AdjLds {
  using TL = Tile<TY>;
  static constexpr int NM = TH ? 9 : 6;
  R r[TL::W2 * TL::H2], vx[TL::W2 * TL::H2], vy[TL::W2 * TL::H2];
  R th[TH ? TL::W2 * TL::H2 : 1], Tn[TH ? TL::W2 * TL::H2 : 1], B[TH ? TL::W2 * TL::H2 : 1];
  R m[NM][TL::W1 * TL::H1];
};

// Stage A1 at an interior node: weighted pull of the level-n+1 equilibria
// f~_i^eq = rho~ + c_i.V and g~_i^eq = Theta from x + c_i (raw coefficients
// in LDS, pitch PR, position pr); returns the moments rho~, U~, s~ (xx, xy,
// yy), T~, q~.
template <typename R, bool TH, int PR>
__device__ inline void adj_pull(const R* lr, const R* lvx, const R* lvy, const R* lth, int pr,
                                R mom[9]) {
  R r = R(0), Ux = R(0), Uy = R(0), sxx = R(0), sxy = R(0), syy = R(0);
  R Tt = R(0), qx = R(0), qy = R(0);
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const int p = pr + CX[q] + CY[q] * PR;
    // rho~ + c_i.V with the zero components left out (a product with a
    // constant 0 is not folded away under IEEE rules)
    R E = lr[p];
    if (CX[q] > 0) E += lvx[p];
    if (CX[q] < 0) E -= lvx[p];
    if (CY[q] > 0) E += lvy[p];
    if (CY[q] < 0) E -= lvy[p];
    const R wE = R(WD[q]) * E;
    r += wE;
    if (CX[q]) Ux += R(CX[q]) * wE;
    if (CY[q]) Uy += R(CY[q]) * wE;
    if (CX[q]) sxx += wE;
    if (CX[q] * CY[q]) sxy += R(CX[q] * CY[q]) * wE;
    if (CY[q]) syy += wE;
    if constexpr (TH) {
      const R wT = R(WD[q]) * lth[p];
      Tt += wT;
      if (CX[q]) qx += R(CX[q]) * wT;
      if (CY[q]) qy += R(CY[q]) * wT;
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

// Stage A1 at node (i, j) of the raw region: the moments of the pulled and,
// on ring nodes, completed adjoint populations, stored at position pm of the
// moment arrays (each field SM values apart). Corners are left to the
// caller.
template <typename R, bool TH, int PR, int SM, bool INT = false>
__device__ inline void adj_moments(const Geo& g, const AdjArgs<R>& a, const R* lr, const R* lvx,
                                   const R* lvy, const R* lth, const R* lTn, int pr, int i,
                                   int j, R* lm, int pm) {
  constexpr int NM = TH ? 9 : 6;
  const bool ring = !INT && !g.periodic && (i == 0 || j == 0 || i == g.nx - 1 || j == g.ny - 1);
  R mom[9];
  if (!ring) {
    adj_pull<R, TH, PR>(lr, lvx, lvy, lth, pr, mom);
  } else {
    const bool corner = (i == 0 || i == g.nx - 1) && (j == 0 || j == g.ny - 1);
    if (corner) return;
    const int k = j * g.nx + i;
    ring_moments<R, TH, PR>(g, a, lr, lvx, lvy, lth, lTn, pr, i, j, k, a.mask[k], mom);
  }
#pragma unroll
  for (int f = 0; f < NM; ++f) lm[f * SM + pm] = mom[f];
}

// corners copy the moments of their y-neighbour; the region of moment
// positions starts at node (rx0, ry0), pitch PM, and spans rw x rh nodes
template <typename R, bool TH, int PM, int SM>
__device__ inline void adj_corners(const Geo& g, R* lm, int rx0, int ry0, int rw, int rh) {
  constexpr int NM = TH ? 9 : 6;
  if (g.periodic || threadIdx.x >= 4) return;
  const int ci = (threadIdx.x & 1) ? g.nx - 1 : 0;
  const int cj = (threadIdx.x & 2) ? g.ny - 1 : 0;
  if (ci < rx0 || ci >= rx0 + rw || cj < ry0 || cj >= ry0 + rh) return;
  const int pm = (cj - ry0) * PM + (ci - rx0);
  const int pn = pm + (cj == 0 ? PM : -PM);
#pragma unroll
  for (int f = 0; f < NM; ++f) lm[f * SM + pm] = lm[f * SM + pn];
}

// Stage B at node (i, j): the local terms of eq:albef_ex / eq:albeg_ex at
// level n (seeds, 3 T q~ coupling, implicit Brinkman), then V and Theta of
// the new level from the moments (pitch PM, position pm) and, when want_sens
// is set, the sensitivity integrand 3 alpha' u.u~ - B' grad T . q~.
template <typename R, bool TH, int PR, int PM, int SM, bool INT = false>
__device__ inline void adj_local(const Geo& g, const AdjArgs<R>& a, const R* lm, int pm,
                                 const R* lTn, const R* lB, int pr, int i, int j, int k, R s,
                                 R ux, R uy, R& r_out, R& Vx, R& Vy, R& Th, bool want_sens,
                                 double& sens) {
  const R A2 = R(2.0 * g.A);
  const bool ring = !INT && !g.periodic && (i == 0 || j == 0 || i == g.nx - 1 || j == g.ny - 1);
  const bool corner = ring && (i == 0 || i == g.nx - 1) && (j == 0 || j == g.ny - 1);
  // local terms are those of the node whose moments were taken
  const int kl = corner ? (j == 0 ? g.nx + i : (g.ny - 2) * g.nx + i) : k;
  const int pl = corner ? pr + (j == 0 ? PR : -PR) : pr;
  const R r = lm[0 * SM + pm];
  R Ux = lm[1 * SM + pm], Uy = lm[2 * SM + pm];
  const R sxx = lm[3 * SM + pm], sxy = lm[4 * SM + pm], syy = lm[5 * SM + pm];
  R Tt = R(0), qx = R(0), qy = R(0);
  if constexpr (TH) {
    Tt = lm[6 * SM + pm];
    qx = lm[7 * SM + pm];
    qy = lm[8 * SM + pm];
    const R Tl = lTn[pl];
    Ux += Tl * qx;
    Uy += Tl * qy;
    if (a.seed_heat != 0.0 && (a.mask[kl] & TAG_PROBE)) {
      Ux -= R(a.seed_heat / 3.0) * Tl;
      Tt -= R(a.seed_heat) * a.ux[kl];
    }
  }
  // paper: u~ = U~ / (1 + alpha) here; exact: V is divided by 1 + alpha
  // instead, after it is formed from the undivided u~
  const R su = a.exact ? R(1) : s;
  const R utx = Ux * su, uty = Uy * su;
  // paper: the Boussinesq coupling of eq:albeg_ex, 3 g beta . u~ on T~ at
  // interior nodes (zero when g beta is zero)
  if constexpr (TH)
    if (!ring && !a.exact) Tt += R(3) * (R(g.gbx) * utx + R(g.gby) * uty);
  // heat source (interior nodes; beta = 0 on the ring): the heat-exchange
  // seed dJ/dg_i = seed_src beta, and in paper mode the implicit
  // T~ (1 + beta) of eq:albeg_ex
  R bsrc = R(0);
  if constexpr (TH) {
    if (a.beta && !ring) {
      bsrc = a.beta[k];
      Tt -= R(a.seed_src) * bsrc;
      if (!a.exact) Tt /= R(1) + bsrc;
    }
  }
  auto ldx = [&](int f) { return lds_dx<INT>(lm + f * SM, pm, 1, i, g.nx, g.periodic); };
  auto ldy = [&](int f) { return lds_dx<INT>(lm + f * SM, pm, PM, j, g.ny, g.periodic); };
  const R dsx = ldx(3) + ldy(4);
  const R dsy = ldx(4) + ldy(5);
  r_out = r;
  Vx = R(3) * utx + R(9) * (sxx * ux + sxy * uy) - R(3) * r * ux - A2 * dsx;
  Vy = R(3) * uty + R(9) * (sxy * ux + syy * uy) - R(3) * r * uy - A2 * dsy;
  // the Brinkman pairing of the sensitivity: 3 alpha' u.u~ (paper) or
  // alpha' u.V / (1 + alpha) with the undivided V (exact)
  const double pair = a.exact ? double(s) / 3.0 * (double(ux) * double(Vx) + double(uy) * double(Vy))
                              : double(ux) * double(utx) + double(uy) * double(uty);
  if (a.exact) {
    Vx *= s;
    Vy *= s;
  }
  if constexpr (TH) {
    if (a.exact) {
      // exact: the transpose of the forward B c.grad_h T, -div_h (B q~)
      const R dbx = lds_dxp<INT>(lB, pr, 1, lm + 7 * SM, pm, 1, i, g.nx, g.periodic);
      const R dby = lds_dxp<INT>(lB, pr, PR, lm + 8 * SM, pm, PM, j, g.ny, g.periodic);
      Th = Tt + R(3) * (qx * ux + qy * uy) - (dbx + dby);
    } else {
      const R divq = ldx(7) + ldy(8);
      const R Bk = lB[pr];
      const R dBx = lds_dx<INT>(lB, pr, 1, i, g.nx, g.periodic);
      const R dBy = lds_dx<INT>(lB, pr, PR, j, g.ny, g.periodic);
      Th = Tt + R(3) * (qx * ux + qy * uy) - Bk * divq - (dBx * qx + dBy * qy);
    }
    // exact: the propagated Theta carries the force's dependence on the new
    // temperature, g beta . V / (1 + alpha), at interior nodes
    if (!ring && a.exact) Th += R(g.gbx) * Vx + R(g.gby) * Vy;
    // exact: the division by 1 + beta acts on the propagated Theta
    if (a.exact && a.beta) Th /= R(1) + bsrc;
  }
  sens = 0.0;
  if (want_sens) {
    double v = 0.0;
    if (!ring) {
      // exact mode at level 0 keeps only the conductivity term: alpha and
      // beta act on the levels the steps produce, B on the equilibria used
      v = a.sens_b_only ? 0.0 : double(a.dA3[k]) * pair;
      if constexpr (TH) {
        const double dTx = double(lds_dx<INT>(lTn, pr, 1, i, g.nx, g.periodic));
        const double dTy = double(lds_dx<INT>(lTn, pr, PR, j, g.ny, g.periodic));
        v -= double(a.dB[k]) * (dTx * double(qx) + dTy * double(qy));
        // heat source and heat-exchange objective: beta' (T - 1)(w_J + T~),
        // with the propagated Theta in exact mode
        if (a.beta && !a.sens_b_only)
          v += double(a.dbeta[k]) * (double(lTn[pr]) - 1.0) *
               (a.seed_src + double(a.exact ? Th : Tt));
      }
    }
    sens = v;
  }
}

template <typename R, bool TH, int TY, bool FULL, int KIND, int NT = NT1<R, TH, TY>>
__device__ void alks_tile(const Geo& g, const AdjArgs<R>& a, AdjLds<R, TH, TY>& L, int x0,
                          int y0, int tw, int th) {
  using TL = Tile<TY>;
  constexpr int W2 = TL::W2, W1 = TL::W1, SM = TL::W1 * TL::H1;
  constexpr bool INT = KIND == K_INT, EDGE = KIND == K_EDGE;
  if constexpr (FULL) {
    tw = TX;
    th = TY;
  }
  // node-local inputs of stage B, loaded before the first barrier (full
  // tiles), the accumulated sensitivity among them: its read-modify-write
  // would otherwise wait for the load at the end of the tile
  constexpr int NB = FULL ? (TX * TY + NT - 1) / NT : 1;
  R spre[NB], uxpre[NB], uypre[NB];
  double senspre[NB];
  if constexpr (FULL) {
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int p = e * NT + int(threadIdx.x);
      if (p >= TX * TY) break;  // more threads than tile nodes
      const int k = (y0 + p / TX) * g.nx + x0 + p % TX;
      spre[e] = a.inv1pa[k];
      uxpre[e] = a.ux[k];
      uypre[e] = a.uy[k];
      senspre[e] = a.sens_mode == 1 ? a.sens[k] : 0.0;
    }
  }

  if constexpr (TH) {
    const R* src[6] = {a.r0, a.vx0, a.vy0, a.th0, a.T, a.B};
    R* dst[6] = {L.r, L.vx, L.vy, L.th, L.Tn, L.B};
    load_halo<R, FULL, TY, 2, W2, 6, INT, NT>(g, x0, y0, tw, th, src, dst);
  } else {
    const R* src[3] = {a.r0, a.vx0, a.vy0};
    R* dst[3] = {L.r, L.vx, L.vy};
    load_halo<R, FULL, TY, 2, W2, 3, INT, NT>(g, x0, y0, tw, th, src, dst);
  }
  __syncthreads();

  region_walk<KIND, FULL, TX + 2, TY + 2, NT>(g, x0, y0, 1, tw + 2, th + 2,
                                          [&](auto in, int lx, int ly, int i, int j) {
    adj_moments<R, TH, W2, SM, decltype(in)::value>(g, a, L.r, L.vx, L.vy, L.th, L.Tn,
                                                    (ly + 1) * W2 + lx + 1, i, j, &L.m[0][0],
                                                    ly * W1 + lx);
  });
  __syncthreads();
  const bool has_corner =
      !INT && !g.periodic && (x0 == 0 || x0 + tw == g.nx) && (y0 == 0 || y0 + th == g.ny);
  if (has_corner) {
    adj_corners<R, TH, W1, SM>(g, &L.m[0][0], x0 - 1, y0 - 1, tw + 2, th + 2);
    __syncthreads();
  }

  // the local terms, new coefficients and sensitivity of node (i, j); sold
  // is the node's accumulated sensitivity when `pre` (else it is read here)
  auto local = [&](auto in, int lx, int ly, int i, int j, R s, R ux, R uy, bool pre,
                   double sold) {
    const int k = j * g.nx + i;
    R r, Vx, Vy, Th;
    double v;
    adj_local<R, TH, W2, W1, SM, decltype(in)::value>(
        g, a, &L.m[0][0], (ly + 1) * W1 + lx + 1, L.Tn, L.B, (ly + 2) * W2 + lx + 2, i, j, k, s,
        ux, uy, r, Vx, Vy, Th, a.sens_mode != 0, v);
    a.r1[k] = r;
    a.vx1[k] = Vx;
    a.vy1[k] = Vy;
    if constexpr (TH) a.th1[k] = Th;
    if (a.sens_mode == 1) a.sens[k] = (pre ? sold : a.sens[k]) + v;
    else if (a.sens_mode == 2) a.sens[k] = v;
  };
  int e = 0;
  rect_loop<FULL, TX, TY, NT>(tw, th, [&](int lx, int ly) {
    const int i = x0 + lx, j = y0 + ly;
    R s, ux, uy;
    double so = 0.0;
    if constexpr (FULL) {
      s = pick(spre, e);
      ux = pick(uxpre, e);
      uy = pick(uypre, e);
      so = pick(senspre, e);
      ++e;
      if constexpr (EDGE)
        if (on_ring(g, i, j)) return;
    } else {
      if constexpr (EDGE)
        if (on_ring(g, i, j)) return;
      const int k = j * g.nx + i;
      s = a.inv1pa[k];
      ux = a.ux[k];
      uy = a.uy[k];
    }
    local(BoolC<INT || EDGE>(), lx, ly, i, j, s, ux, uy, FULL, so);
  });
  if constexpr (EDGE)
    ring_loop<NT>(g, x0, y0, tw, th, [&](int i, int j) {
      const int k = j * g.nx + i;
      local(BoolC<false>(), i - x0, j - y0, i, j, a.inv1pa[k], a.ux[k], a.uy[k], false, 0.0);
    });
}

template <typename R, bool TH, int TY>
__global__ __launch_bounds__((NT1<R, TH, TY>)) void alks_step_kernel(Geo g, AdjArgs<R> a) {
  __shared__ AdjLds<R, TH, TY> L;
  int x0, x1, y0, y1, tile;
  if (!block_tile(g, &x0, &x1, &y0, &y1, &tile)) return;
  const int tw = x1 - x0, th = y1 - y0;
  if (tw != TX || th != TY) {
    if (g.periodic) alks_tile<R, TH, TY, false, K_GEN>(g, a, L, x0, y0, tw, th);
    else alks_tile<R, TH, TY, false, K_EDGE>(g, a, L, x0, y0, tw, th);
  } else if (interior_tile(g, x0, x1, y0, y1)) {
    alks_tile<R, TH, TY, true, K_INT>(g, a, L, x0, y0, tw, th);
  } else if (g.periodic) {
    alks_tile<R, TH, TY, false, K_GEN>(g, a, L, x0, y0, tw, th);
  } else {
    alks_tile<R, TH, TY, true, K_EDGE>(g, a, L, x0, y0, tw, th);
  }
}

// ---------------------------------------------------------------------------
// two steps per launch (steady sweeps)
// ---------------------------------------------------------------------------
// Temporal blocking: a block loads the raw state of its tile with a 4-node
// halo once, runs the first step on the tile and a 2-node halo into LDS and
// the second step on the tile into HBM. Each node's arithmetic is that of
// the one-step kernel (the same stage functions), so two fused steps give
// the same bits as two single steps; the launch count and the global
// round trips per step halve, the stage work grows by the halo (about 1.3x
// for 64 x 8 tiles).
// threads of a two-step block: the stages walk tile + 3, + 2 and + 1 regions of
// up to 3.4x the tile's nodes, so a block of 512 threads (8 waves) keeps each
// stage to one or two passes
template <bool TH>
constexpr int NT2 = 512;

template <typename R, bool TH, int TY>
struct Fwd2Lds {
  static constexpr int WR = TX + 1 + 8, HR = TY + 1 + 8;  // raw state: tile + 4
  static constexpr int WF = TX + 1 + 6, HF = TY + 1 + 6;  // post-collision: tile + 3
  static constexpr int SF = WF * HF;
  R d[WR * HR], u[WR * HR], v[WR * HR];
  R T[TH ? WR * HR : 1], B[TH ? WR * HR : 1];
  R f[9 * SF];
  R gq[TH ? 2 * SF : 1];
  // T of the intermediate level: the first pull rewrites drho and u in place
  // but still reads the sources' T, so the new T goes beside it
  R T2[TH ? WR * HR : 1];
  double red[8];
};

template <typename R, bool TH, int TY, bool FULL, int KIND, int NT>
__device__ __forceinline__ void lks_tile2(const Geo& g, const FwdArgs<R>& a, Fwd2Lds<R, TH, TY>& L, int x0,
                          int y0, int tw, int th, int tile) {
  using LD = Fwd2Lds<R, TH, TY>;
  constexpr int WR = LD::WR, WF = LD::WF, SF = LD::SF;
  constexpr bool INT = KIND == K_INT, EDGE = KIND == K_EDGE;
  const R A = R(g.A);
  if constexpr (FULL) {
    tw = TX;
    th = TY;
  }
  constexpr int NB = FULL ? (TX * TY + NT - 1) / NT : 1;
  int mpre[NB];
  R spre[NB];
  if constexpr (FULL) {
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int p = e * NT + int(threadIdx.x);
      if (p >= TX * TY) break;  // more threads than tile nodes
      const int k = (y0 + p / TX) * g.nx + x0 + p % TX;
      mpre[e] = a.mask[k];
      spre[e] = a.inv1pa[k];
    }
  }
  if constexpr (TH) {
    const R* src[5] = {a.d0, a.ux0, a.uy0, a.T0, a.B};
    R* dst[5] = {L.d, L.u, L.v, L.T, L.B};
    load_halo<R, FULL, TY, 4, WR, 5, INT, NT>(g, x0, y0, tw, th, src, dst);
  } else {
    const R* src[3] = {a.d0, a.ux0, a.uy0};
    R* dst[3] = {L.d, L.u, L.v};
    load_halo<R, FULL, TY, 4, WR, 3, INT, NT>(g, x0, y0, tw, th, src, dst);
  }
  __syncthreads();
  // first step: collide on the tile + 3, pull on the tile + 2 into LDS
  region_walk<KIND, FULL, TX + 6, TY + 6, NT>(g, x0, y0, 3, tw + 6, th + 6,
                                          [&](auto in, int lx, int ly, int i, int j) {
    fwd_collide<R, TH, WR, SF, decltype(in)::value>(g, A, L.d, L.u, L.v, L.T, L.B,
                                                    (ly + 1) * WR + lx + 1, i, j, L.f, L.gq,
                                                    ly * WF + lx);
  });
  __syncthreads();
  region_walk<KIND, FULL, TX + 4, TY + 4, NT>(g, x0, y0, 2, tw + 4, th + 4,
                                          [&](auto in, int lx, int ly, int i, int j) {
    constexpr bool I = decltype(in)::value;
    const int k = j * g.nx + i;
    const int m = I ? 0 : int(a.mask[k]);
    if (!I && !g.periodic && (m & 3) == FLOW_CORNER) return;
    R dn, uxn, uyn, Tn;
    fwd_pull<R, TH, WF, SF, WR, I>(g, a, L.f, L.gq, L.T, (ly + 1) * WF + lx + 1,
                                   (ly + 2) * WR + lx + 2, i, j, k, m, a.inv1pa[k], a.level_mid,
                                   dn, uxn, uyn, Tn);
    const int pr = (ly + 2) * WR + lx + 2;
    if constexpr (!I)
      corner_from(g, i, j, [&](int jc) {
        const int pc = pr + (jc == 0 ? -WR : WR);
        L.d[pc] = dn;
        L.u[pc] = R(0);
        L.v[pc] = R(0);
        if constexpr (TH) L.T2[pc] = Tn;
      });
    L.d[pr] = dn;
    L.u[pr] = uxn;
    L.v[pr] = uyn;
    if constexpr (TH) L.T2[pr] = Tn;
  });
  __syncthreads();
  // the first step's level on the tile: kept where wanted (corner nodes
  // included), and its objective term (corner nodes excluded, as in the pull)
  if (a.uxm || a.acc) {
    double pm = 0.0;
    auto mid = [&](int lx, int ly, int i, int j) {
      const int k = j * g.nx + i;
      const int pr = (ly + 4) * WR + lx + 4;  // tile position in the tile + 4 region
      const R dn = L.d[pr], uxn = L.u[pr], uyn = L.v[pr];
      const R Tn = TH ? L.T2[pr] : R(0);
      if (a.uxm) {
        if (a.dm) a.dm[k] = dn;
        a.uxm[k] = uxn;
        a.uym[k] = uyn;
        if constexpr (TH) a.Tm[k] = Tn;
      }
      if (a.acc) {
        const int m = a.mask[k];
        if (g.periodic || (m & 3) != FLOW_CORNER) obj_add<R, TH>(a, m, k, dn, uxn, Tn, pm);
      }
    };
    rect_loop<FULL, TX, TY, NT>(tw, th, [&](int lx, int ly) {
      const int i = x0 + lx, j = y0 + ly;
      if constexpr (EDGE)
        if (on_ring(g, i, j)) return;
      mid(lx, ly, i, j);
    });
    if constexpr (EDGE)
      ring_loop<NT>(g, x0, y0, tw, th, [&](int i, int j) { mid(i - x0, j - y0, i, j); });
    if (a.acc) {
      const double sm = block_sum<NT>(pm, L.red);
      if (threadIdx.x == 0) a.acc[tile] += sm;
    }
  }
  // second step: collide on the tile + 1, pull on the tile into HBM
  region_walk<KIND, FULL, TX + 2, TY + 2, NT>(g, x0, y0, 1, tw + 2, th + 2,
                                          [&](auto in, int lx, int ly, int i, int j) {
    fwd_collide<R, TH, WR, SF, decltype(in)::value>(g, A, L.d, L.u, L.v, L.T2, L.B,
                                                    (ly + 3) * WR + lx + 3, i, j, L.f, L.gq,
                                                    (ly + 2) * WF + lx + 2);
  });
  __syncthreads();
  double part = 0.0;
  auto pull = [&](auto in, int lx, int ly, int i, int j, int m, R s) {
    constexpr bool I = decltype(in)::value;
    const int k = j * g.nx + i;
    if (!I && !g.periodic && (m & 3) == FLOW_CORNER) return;
    R dn, uxn, uyn, Tn;
    fwd_pull<R, TH, WF, SF, WR, I>(g, a, L.f, L.gq, L.T2, (ly + 3) * WF + lx + 3,
                                   (ly + 4) * WR + lx + 4, i, j, k, m, s, a.level_out, dn, uxn,
                                   uyn, Tn);
    if constexpr (!I)
      corner_from(g, i, j, [&](int jc) {
        const int kc = jc * g.nx + i;
        a.d1[kc] = dn;
        a.ux1[kc] = R(0);
        a.uy1[kc] = R(0);
        if constexpr (TH) a.T1[kc] = Tn;
      });
    a.d1[k] = dn;
    a.ux1[k] = uxn;
    a.uy1[k] = uyn;
    if constexpr (TH) a.T1[k] = Tn;
    if (a.acc) obj_add<R, TH>(a, m, k, dn, uxn, Tn, part);
  };
  int e = 0;
  rect_loop<FULL, TX, TY, NT>(tw, th, [&](int lx, int ly) {
    const int i = x0 + lx, j = y0 + ly;
    int m;
    R s;
    if constexpr (FULL) {
      m = mpre[e];
      s = spre[e];
      ++e;
      if constexpr (EDGE)
        if (on_ring(g, i, j)) return;
    } else {
      if constexpr (EDGE)
        if (on_ring(g, i, j)) return;
      const int k = j * g.nx + i;
      m = a.mask[k];
      s = a.inv1pa[k];
    }
    pull(BoolC<INT || EDGE>(), lx, ly, i, j, m, s);
  });
  if constexpr (EDGE)
    ring_loop<NT>(g, x0, y0, tw, th, [&](int i, int j) {
      const int k = j * g.nx + i;
      pull(BoolC<false>(), i - x0, j - y0, i, j, int(a.mask[k]), a.inv1pa[k]);
    });
  if (a.acc) {
    const double s = block_sum<NT>(part, L.red);
    if (threadIdx.x == 0) a.acc[tile] += s;
  }
}

template <typename R, bool TH, int TY>
__global__ __launch_bounds__(NT2<TH>) void lks_step2_kernel(Geo g, FwdArgs<R> a) {
  __shared__ Fwd2Lds<R, TH, TY> L;
  int x0, x1, y0, y1, tile;
  if (!block_tile(g, &x0, &x1, &y0, &y1, &tile)) return;
  const int tw = x1 - x0, th = y1 - y0;
  if (tw != TX || th != TY) {
    if (g.periodic) lks_tile2<R, TH, TY, false, K_GEN, NT2<TH>>(g, a, L, x0, y0, tw, th, tile);
    else lks_tile2<R, TH, TY, false, K_EDGE, NT2<TH>>(g, a, L, x0, y0, tw, th, tile);
  } else if (interior_tile2(g, x0, x1, y0, y1)) {
    lks_tile2<R, TH, TY, true, K_INT, NT2<TH>>(g, a, L, x0, y0, tw, th, tile);
  } else if (g.periodic) {
    lks_tile2<R, TH, TY, false, K_GEN, NT2<TH>>(g, a, L, x0, y0, tw, th, tile);
  } else {
    lks_tile2<R, TH, TY, true, K_EDGE, NT2<TH>>(g, a, L, x0, y0, tw, th, tile);
  }
}

template <typename R, bool TH, int TY>
struct Adj2Lds {
  static constexpr int WR = TX + 1 + 8, HR = TY + 1 + 8;  // raw coefficients: tile + 4
  static constexpr int WM = TX + 1 + 6, HM = TY + 1 + 6;  // moments: tile + 3
  static constexpr int SM = WM * HM;
  static constexpr int NM = TH ? 9 : 6;
  R r[WR * HR], vx[WR * HR], vy[WR * HR];
  R th[TH ? WR * HR : 1], Tn[TH ? WR * HR : 1], B[TH ? WR * HR : 1];
  R m[NM * SM];
};

template <typename R, bool TH, int TY, bool FULL, int KIND, int NT>
__device__ __forceinline__ void alks_tile2(const Geo& g, const AdjArgs<R>& a, Adj2Lds<R, TH, TY>& L, int x0,
                           int y0, int tw, int th) {
  using LD = Adj2Lds<R, TH, TY>;
  constexpr int WR = LD::WR, WM = LD::WM, SM = LD::SM;
  constexpr bool INT = KIND == K_INT, EDGE = KIND == K_EDGE;
  if constexpr (FULL) {
    tw = TX;
    th = TY;
  }
  constexpr int NB = FULL ? (TX * TY + NT - 1) / NT : 1;
  R spre[NB], uxpre[NB], uypre[NB];
  if constexpr (FULL) {
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int p = e * NT + int(threadIdx.x);
      if (p >= TX * TY) break;  // more threads than tile nodes
      const int k = (y0 + p / TX) * g.nx + x0 + p % TX;
      spre[e] = a.inv1pa[k];
      uxpre[e] = a.ux[k];
      uypre[e] = a.uy[k];
    }
  }
  if constexpr (TH) {
    const R* src[6] = {a.r0, a.vx0, a.vy0, a.th0, a.T, a.B};
    R* dst[6] = {L.r, L.vx, L.vy, L.th, L.Tn, L.B};
    load_halo<R, FULL, TY, 4, WR, 6, INT, NT>(g, x0, y0, tw, th, src, dst);
  } else {
    const R* src[3] = {a.r0, a.vx0, a.vy0};
    R* dst[3] = {L.r, L.vx, L.vy};
    load_halo<R, FULL, TY, 4, WR, 3, INT, NT>(g, x0, y0, tw, th, src, dst);
  }
  __syncthreads();
  const bool near_corner = !INT && !g.periodic && (x0 <= 3 || x0 + tw + 3 >= g.nx) &&
                           (y0 <= 3 || y0 + th + 3 >= g.ny);
  // first step: moments on the tile + 3, new coefficients on the tile + 2
  region_walk<KIND, FULL, TX + 6, TY + 6, NT>(g, x0, y0, 3, tw + 6, th + 6,
                                          [&](auto in, int lx, int ly, int i, int j) {
    adj_moments<R, TH, WR, SM, decltype(in)::value>(g, a, L.r, L.vx, L.vy, L.th, L.Tn,
                                                    (ly + 1) * WR + lx + 1, i, j, L.m,
                                                    ly * WM + lx);
  });
  __syncthreads();
  if (near_corner) {
    adj_corners<R, TH, WM, SM>(g, L.m, x0 - 3, y0 - 3, tw + 6, th + 6);
    __syncthreads();
  }
  region_walk<KIND, FULL, TX + 4, TY + 4, NT>(g, x0, y0, 2, tw + 4, th + 4,
                                          [&](auto in, int lx, int ly, int i, int j) {
    const int k = j * g.nx + i;
    R r, Vx, Vy, Th;
    double v;
    const int pr = (ly + 2) * WR + lx + 2;
    adj_local<R, TH, WR, WM, SM, decltype(in)::value>(g, a, L.m, (ly + 1) * WM + lx + 1, L.Tn,
                                                      L.B, pr, i, j, k, a.inv1pa[k], a.ux[k],
                                                      a.uy[k], r, Vx, Vy, Th, false, v);
    L.r[pr] = r;
    L.vx[pr] = Vx;
    L.vy[pr] = Vy;
    if constexpr (TH) L.th[pr] = Th;
  });
  __syncthreads();
  // second step: moments on the tile + 1, new coefficients on the tile
  region_walk<KIND, FULL, TX + 2, TY + 2, NT>(g, x0, y0, 1, tw + 2, th + 2,
                                          [&](auto in, int lx, int ly, int i, int j) {
    adj_moments<R, TH, WR, SM, decltype(in)::value>(g, a, L.r, L.vx, L.vy, L.th, L.Tn,
                                                    (ly + 3) * WR + lx + 3, i, j, L.m,
                                                    (ly + 2) * WM + lx + 2);
  });
  __syncthreads();
  if (near_corner) {
    adj_corners<R, TH, WM, SM>(g, L.m + 2 * WM + 2, x0 - 1, y0 - 1, tw + 2, th + 2);
    __syncthreads();
  }
  auto local = [&](auto in, int lx, int ly, int i, int j, R s, R ux, R uy) {
    const int k = j * g.nx + i;
    R r, Vx, Vy, Th;
    double v;
    adj_local<R, TH, WR, WM, SM, decltype(in)::value>(
        g, a, L.m, (ly + 3) * WM + lx + 3, L.Tn, L.B, (ly + 4) * WR + lx + 4, i, j, k, s, ux, uy,
        r, Vx, Vy, Th, a.sens_mode != 0, v);
    a.r1[k] = r;
    a.vx1[k] = Vx;
    a.vy1[k] = Vy;
    if constexpr (TH) a.th1[k] = Th;
    if (a.sens_mode == 1) a.sens[k] += v;
    else if (a.sens_mode == 2) a.sens[k] = v;
  };
  int e = 0;
  rect_loop<FULL, TX, TY, NT>(tw, th, [&](int lx, int ly) {
    const int i = x0 + lx, j = y0 + ly;
    R s, ux, uy;
    if constexpr (FULL) {
      s = spre[e];
      ux = uxpre[e];
      uy = uypre[e];
      ++e;
      if constexpr (EDGE)
        if (on_ring(g, i, j)) return;
    } else {
      if constexpr (EDGE)
        if (on_ring(g, i, j)) return;
      const int k = j * g.nx + i;
      s = a.inv1pa[k];
      ux = a.ux[k];
      uy = a.uy[k];
    }
    local(BoolC<INT || EDGE>(), lx, ly, i, j, s, ux, uy);
  });
  if constexpr (EDGE)
    ring_loop<NT>(g, x0, y0, tw, th, [&](int i, int j) {
      const int k = j * g.nx + i;
      local(BoolC<false>(), i - x0, j - y0, i, j, a.inv1pa[k], a.ux[k], a.uy[k]);
    });
}

template <typename R, bool TH, int TY>
__global__ __launch_bounds__(NT2<TH>) void alks_step2_kernel(Geo g, AdjArgs<R> a) {
  __shared__ Adj2Lds<R, TH, TY> L;
  int x0, x1, y0, y1, tile;
  if (!block_tile(g, &x0, &x1, &y0, &y1, &tile)) return;
  const int tw = x1 - x0, th = y1 - y0;
  if (tw != TX || th != TY) {
    if (g.periodic) alks_tile2<R, TH, TY, false, K_GEN, NT2<TH>>(g, a, L, x0, y0, tw, th);
    else alks_tile2<R, TH, TY, false, K_EDGE, NT2<TH>>(g, a, L, x0, y0, tw, th);
  } else if (interior_tile2(g, x0, x1, y0, y1)) {
    alks_tile2<R, TH, TY, true, K_INT, NT2<TH>>(g, a, L, x0, y0, tw, th);
  } else if (g.periodic) {
    alks_tile2<R, TH, TY, false, K_GEN, NT2<TH>>(g, a, L, x0, y0, tw, th);
  } else {
    alks_tile2<R, TH, TY, true, K_EDGE, NT2<TH>>(g, a, L, x0, y0, tw, th);
  }
}

// ---------------------------------------------------------------------------
// batched steps: many independent designs in one launch
// ---------------------------------------------------------------------------
// Block b runs global tile xcd_tile(total); the host-built table tmap holds,
// for every global tile, its design and its tile index within the design.
// All designs advance in lockstep, so one parity selects the ping-pong
// buffers of every design.
// the tile lt of design g in the rule its kind takes (as the one-design
// step launch does, so a design gives the same bits alone and in a batch)
template <typename R, bool TH, int TY>
__device__ inline void batch_fwd_tile(const Geo& g, const FwdArgs<R>& a, FwdLds<R, TH, TY>& L,
                                      int lt) {
  int x0, x1, y0, y1;
  tile_box(g, lt, &x0, &x1, &y0, &y1);
  const int tw = x1 - x0, th = y1 - y0;
  if (tw != TX || th != TY) {
    if (g.periodic) lks_tile<R, TH, TY, false, K_GEN>(g, a, L, x0, y0, tw, th, lt);
    else lks_tile<R, TH, TY, false, K_EDGE>(g, a, L, x0, y0, tw, th, lt);
  } else if (interior_tile(g, x0, x1, y0, y1)) {
    lks_tile<R, TH, TY, true, K_INT>(g, a, L, x0, y0, tw, th, lt);
  } else if (g.periodic) {
    lks_tile<R, TH, TY, false, K_GEN>(g, a, L, x0, y0, tw, th, lt);
  } else {
    lks_tile<R, TH, TY, true, K_EDGE>(g, a, L, x0, y0, tw, th, lt);
  }
}

template <typename R, bool TH, int TY>
__device__ inline void batch_adj_tile(const Geo& g, const AdjArgs<R>& a, AdjLds<R, TH, TY>& L,
                                      int lt) {
  int x0, x1, y0, y1;
  tile_box(g, lt, &x0, &x1, &y0, &y1);
  const int tw = x1 - x0, th = y1 - y0;
  if (tw != TX || th != TY) {
    if (g.periodic) alks_tile<R, TH, TY, false, K_GEN>(g, a, L, x0, y0, tw, th);
    else alks_tile<R, TH, TY, false, K_EDGE>(g, a, L, x0, y0, tw, th);
  } else if (interior_tile(g, x0, x1, y0, y1)) {
    alks_tile<R, TH, TY, true, K_INT>(g, a, L, x0, y0, tw, th);
  } else if (g.periodic) {
    alks_tile<R, TH, TY, false, K_GEN>(g, a, L, x0, y0, tw, th);
  } else {
    alks_tile<R, TH, TY, true, K_EDGE>(g, a, L, x0, y0, tw, th);
  }
}

template <typename R, bool TH, int TY>
__global__ __launch_bounds__((NT1<R, TH, TY>)) void lks_step_batch_kernel(const BatchFwd<R>* __restrict__ d,
                                                                  const int* __restrict__ tmap,
                                                                  int total, int parity) {
  __shared__ FwdLds<R, TH, TY> L;
  const int t = xcd_tile(total);
  if (t < 0) return;
  const int di = tmap[2 * t];
  const Geo g = d[di].g;
  const FwdArgs<R> a = d[di].a[parity];
  batch_fwd_tile<R, TH, TY>(g, a, L, tmap[2 * t + 1]);
}

template <typename R, bool TH, int TY>
__global__ __launch_bounds__((NT1<R, TH, TY>)) void alks_step_batch_kernel(const BatchAdj<R>* __restrict__ d,
                                                                   const int* __restrict__ tmap,
                                                                   int total, int parity,
                                                                   int last) {
  __shared__ AdjLds<R, TH, TY> L;
  const int t = xcd_tile(total);
  if (t < 0) return;
  const int di = tmap[2 * t];
  const Geo g = d[di].g;
  AdjArgs<R> a = d[di].a[parity];
  a.sens_mode = last ? 2 : 0;
  batch_adj_tile<R, TH, TY>(g, a, L, tmap[2 * t + 1]);
}

// unsteady batches: the level pointers of every design resolved from its
// store (the descriptors' parity-0 arguments give everything else)
template <typename R, bool TH, int TY>
__global__ __launch_bounds__((NT1<R, TH, TY>)) void lks_step_ubatch_kernel(
    const BatchFwd<R>* __restrict__ d, const BatchStore<R>* __restrict__ st,
    const int* __restrict__ tmap, int total, LevelRef in, LevelRef out, int level_out,
    int use_acc) {
  __shared__ FwdLds<R, TH, TY> L;
  const int t = xcd_tile(total);
  if (t < 0) return;
  const int di = tmap[2 * t];
  const BatchStore<R> s = st[di];
  const Geo g = d[di].g;
  FwdArgs<R> a = d[di].a[0];
  a.d0 = level_field(s, in, 0);
  a.ux0 = level_field(s, in, 1);
  a.uy0 = level_field(s, in, 2);
  a.T0 = level_field(s, in, 3);
  a.d1 = level_field(s, out, 0);
  a.ux1 = level_field(s, out, 1);
  a.uy1 = level_field(s, out, 2);
  a.T1 = level_field(s, out, 3);
  a.level_out = level_out < s.n_ufac - 1 ? level_out : s.n_ufac - 1;
  if (!use_acc) a.acc = nullptr;
  batch_fwd_tile<R, TH, TY>(g, a, L, tmap[2 * t + 1]);
}

template <typename R, bool TH, int TY>
__global__ __launch_bounds__((NT1<R, TH, TY>)) void alks_step_ubatch_kernel(
    const BatchAdj<R>* __restrict__ d, const BatchStore<R>* __restrict__ st,
    const int* __restrict__ tmap, int total, int parity, LevelRef lv, int seeded, int b_only) {
  __shared__ AdjLds<R, TH, TY> L;
  const int t = xcd_tile(total);
  if (t < 0) return;
  const int di = tmap[2 * t];
  const BatchStore<R> s = st[di];
  const Geo g = d[di].g;
  AdjArgs<R> a = d[di].a[parity];
  a.ux = level_field(s, lv, 1);
  a.uy = level_field(s, lv, 2);
  const R* T = level_field(s, lv, 3);
  a.T = T ? T : a.ux;
  a.sens_mode = 1;
  if (!seeded) {
    a.seed_dp = 0.0;
    a.seed_heat = 0.0;
  }
  a.sens_b_only = b_only;
  batch_adj_tile<R, TH, TY>(g, a, L, tmap[2 * t + 1]);
}

// per-tile objective accumulators of every design: zeroed, and summed in the
// order of sum_kernel (one block per design)
template <typename R>
__global__ __launch_bounds__(NTHREADS) void acc_zero_batch_kernel(const BatchFwd<R>* d) {
  const Geo& g = d[blockIdx.x].g;
  double* acc = d[blockIdx.x].a[0].acc;
  for (int t = threadIdx.x; t < g.ntx * g.nty; t += NTHREADS) acc[t] = 0.0;
}
template <typename R>
__global__ __launch_bounds__(NTHREADS) void acc_sum_batch_kernel(const BatchFwd<R>* d,
                                                                 double* out) {
  __shared__ double red[NTHREADS / 64];
  const Geo& g = d[blockIdx.x].g;
  const double* v = d[blockIdx.x].a[0].acc;
  const int n = g.ntx * g.nty;
  double part = 0.0;
  for (int t = threadIdx.x; t < n; t += NTHREADS) part += v[t];
  double s = block_sum(part, red);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// pressure drop of every design on its current level: one block per design
template <typename R>
__global__ __launch_bounds__(NTHREADS) void pressure_drop_batch_kernel(const BatchFwd<R>* d,
                                                                      int parity, double* out) {
  __shared__ double red[NTHREADS / 64];
  const Geo g = d[blockIdx.x].g;
  const FwdArgs<R>& a = d[blockIdx.x].a[parity];
  const int per = 2 * g.nx + 2 * g.ny;
  double part = 0.0;
  for (int t = threadIdx.x; t < per; t += NTHREADS) {
    int i, j;
    if (t < g.nx) { i = t; j = 0; }
    else if (t < 2 * g.nx) { i = t - g.nx; j = g.ny - 1; }
    else if (t < 2 * g.nx + g.ny) { i = 0; j = t - 2 * g.nx; }
    else { i = g.nx - 1; j = t - 2 * g.nx - g.ny; }
    const int k = j * g.nx + i;
    const int m = a.mask[k];
    if ((m & 3) == FLOW_CORNER) continue;
    if (m & TAG_J_INLET) part += double(a.d0[k]);
    if (m & TAG_J_OUTLET) part -= double(a.d0[k]);
  }
  double s = block_sum(part, red);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
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

// sum of T over the probe-tagged nodes (heat-sink objective, before the mean)
template <typename R>
__global__ __launch_bounds__(NTHREADS) void probe_T_kernel(Geo g, const uint8_t* mask, const R* T,
                                                          double* out) {
  __shared__ double red[NTHREADS / 64];
  double part = 0.0;
  for (int k = threadIdx.x; k < g.N; k += NTHREADS)
    if (mask[k] & TAG_PROBE) part += double(T[k]);
  double s = block_sum(part, red);
  if (threadIdx.x == 0) *out = s;
}

// sum of beta (T - 1) over all nodes: the heat-exchange objective
// -sum beta (1 - T) of one level
template <typename R>
__global__ __launch_bounds__(NTHREADS) void source_heat_kernel(Geo g, const R* beta, const R* T,
                                                              double* out) {
  __shared__ double red[NTHREADS / 64];
  double part = 0.0;
  for (int k = threadIdx.x; k < g.N; k += NTHREADS)
    part += double(beta[k]) * (double(T[k]) - 1.0);
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
void launch_source_coef(const Geo& g, const double* gamma, double bmax, double qb, R* beta,
                        R* dbeta, hipStream_t s) {
  source_coef_kernel<R><<<blocks_for(g.N), 256, 0, s>>>(g, gamma, bmax, qb, beta, dbeta);
}
template <typename R>
void launch_init(const Geo& g, const uint8_t* mask, const R* ubx, const R* uby, const R* Tb,
                 double fac0, R* d, R* ux, R* uy, R* T, hipStream_t s) {
  init_kernel<R><<<blocks_for(g.N), 256, 0, s>>>(g, mask, ubx, uby, Tb, fac0, d, ux, uy, T);
}
template <typename R>
void launch_lks_step(const Geo& g, const FwdArgs<R>& a, hipStream_t s) {
  const unsigned nb = unsigned(xcd_blocks(g.ntx * g.nty));
  if constexpr (std::is_same<R, float>::value) {
    if (g.ty == 16 && !g.thermal) {
      lks_step_kernel<float, false, 16><<<nb, (NT1<float, false, 16>), 0, s>>>(g, a);
      return;
    }
  }
  if (g.ty == 8) {
    if (g.thermal) lks_step_kernel<R, true, 8><<<nb, (NT1<R, true, 8>), 0, s>>>(g, a);
    else lks_step_kernel<R, false, 8><<<nb, (NT1<R, false, 8>), 0, s>>>(g, a);
  } else {
    if (g.thermal) lks_step_kernel<R, true, 4><<<nb, (NT1<R, true, 4>), 0, s>>>(g, a);
    else lks_step_kernel<R, false, 4><<<nb, (NT1<R, false, 4>), 0, s>>>(g, a);
  }
}
template <typename R>
void launch_alks_step(const Geo& g, const AdjArgs<R>& a, hipStream_t s) {
  const unsigned nb = unsigned(xcd_blocks(g.ntx * g.nty));
  if constexpr (std::is_same<R, float>::value) {
    if (g.ty == 16 && !g.thermal) {
      alks_step_kernel<float, false, 16><<<nb, (NT1<float, false, 16>), 0, s>>>(g, a);
      return;
    }
  }
  if (g.ty == 8) {
    if (g.thermal) alks_step_kernel<R, true, 8><<<nb, (NT1<R, true, 8>), 0, s>>>(g, a);
    else alks_step_kernel<R, false, 8><<<nb, (NT1<R, false, 8>), 0, s>>>(g, a);
  } else {
    if (g.thermal) alks_step_kernel<R, true, 4><<<nb, (NT1<R, true, 4>), 0, s>>>(g, a);
    else alks_step_kernel<R, false, 4><<<nb, (NT1<R, false, 4>), 0, s>>>(g, a);
  }
}
// two-step kernels exist for tile heights 4 and 8 (the runtime never asks for others)
void launch_lks_step2(const Geo& g, const FwdArgs<float>& a, hipStream_t s) {
  const unsigned nb = unsigned(xcd_blocks(g.ntx * g.nty));
  if (g.thermal) {
    if (g.ty == 8) lks_step2_kernel<float, true, 8><<<nb, NT2<true>, 0, s>>>(g, a);
    else lks_step2_kernel<float, true, 4><<<nb, NT2<true>, 0, s>>>(g, a);
  } else {
    if (g.ty == 8) lks_step2_kernel<float, false, 8><<<nb, NT2<false>, 0, s>>>(g, a);
    else lks_step2_kernel<float, false, 4><<<nb, NT2<false>, 0, s>>>(g, a);
  }
}
// FP64: the non-thermal forward step (its LDS, 79 KB at 64 x 4 and 106 KB at
// 64 x 8, leaves room for one or two blocks per CU)
void launch_lks_step2(const Geo& g, const FwdArgs<double>& a, hipStream_t s) {
  const unsigned nb = unsigned(xcd_blocks(g.ntx * g.nty));
  if (g.ty == 8) lks_step2_kernel<double, false, 8><<<nb, NT2<false>, 0, s>>>(g, a);
  else lks_step2_kernel<double, false, 4><<<nb, NT2<false>, 0, s>>>(g, a);
}
void launch_alks_step2(const Geo& g, const AdjArgs<float>& a, hipStream_t s) {
  const unsigned nb = unsigned(xcd_blocks(g.ntx * g.nty));
  if (g.thermal) {
    if (g.ty == 8) alks_step2_kernel<float, true, 8><<<nb, NT2<true>, 0, s>>>(g, a);
    else alks_step2_kernel<float, true, 4><<<nb, NT2<true>, 0, s>>>(g, a);
  } else {
    if (g.ty == 8) alks_step2_kernel<float, false, 8><<<nb, NT2<false>, 0, s>>>(g, a);
    else alks_step2_kernel<float, false, 4><<<nb, NT2<false>, 0, s>>>(g, a);
  }
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
template <typename R>
void launch_probe_T(const Geo& g, const uint8_t* mask, const R* T, double* out, hipStream_t s) {
  probe_T_kernel<R><<<1, NTHREADS, 0, s>>>(g, mask, T, out);
}
template <typename R>
void launch_source_heat(const Geo& g, const R* beta, const R* T, double* out, hipStream_t s) {
  source_heat_kernel<R><<<1, NTHREADS, 0, s>>>(g, beta, T, out);
}
template <typename R>
void launch_lks_step_batch(const BatchFwd<R>* d, const int* tmap, int total, int ty,
                           bool thermal, int parity, hipStream_t s) {
  const unsigned nb = unsigned(xcd_blocks(total));
  if constexpr (std::is_same<R, float>::value) {
    if (ty == 16 && !thermal) {
      lks_step_batch_kernel<float, false, 16><<<nb, (NT1<float, false, 16>), 0, s>>>(d, tmap, total, parity);
      return;
    }
  }
  if (ty == 8) {
    if (thermal) lks_step_batch_kernel<R, true, 8><<<nb, (NT1<R, true, 8>), 0, s>>>(d, tmap, total, parity);
    else lks_step_batch_kernel<R, false, 8><<<nb, (NT1<R, false, 8>), 0, s>>>(d, tmap, total, parity);
  } else {
    if (thermal) lks_step_batch_kernel<R, true, 4><<<nb, (NT1<R, true, 4>), 0, s>>>(d, tmap, total, parity);
    else lks_step_batch_kernel<R, false, 4><<<nb, (NT1<R, false, 4>), 0, s>>>(d, tmap, total, parity);
  }
}
template <typename R>
void launch_alks_step_batch(const BatchAdj<R>* d, const int* tmap, int total, int ty,
                            bool thermal, int parity, int last, hipStream_t s) {
  const unsigned nb = unsigned(xcd_blocks(total));
  if constexpr (std::is_same<R, float>::value) {
    if (ty == 16 && !thermal) {
      alks_step_batch_kernel<float, false, 16><<<nb, (NT1<float, false, 16>), 0, s>>>(d, tmap, total, parity,
                                                                       last);
      return;
    }
  }
  if (ty == 8) {
    if (thermal) alks_step_batch_kernel<R, true, 8><<<nb, (NT1<R, true, 8>), 0, s>>>(d, tmap, total, parity, last);
    else alks_step_batch_kernel<R, false, 8><<<nb, (NT1<R, false, 8>), 0, s>>>(d, tmap, total, parity, last);
  } else {
    if (thermal) alks_step_batch_kernel<R, true, 4><<<nb, (NT1<R, true, 4>), 0, s>>>(d, tmap, total, parity, last);
    else alks_step_batch_kernel<R, false, 4><<<nb, (NT1<R, false, 4>), 0, s>>>(d, tmap, total, parity, last);
  }
}
template <typename R>
void launch_pressure_drop_batch(const BatchFwd<R>* d, int nd, int parity, double* out,
                                hipStream_t s) {
  pressure_drop_batch_kernel<R><<<nd, NTHREADS, 0, s>>>(d, parity, out);
}
template <typename R>
void launch_lks_step_ubatch(const BatchFwd<R>* d, const BatchStore<R>* st, const int* tmap,
                            int total, int ty, bool thermal, LevelRef in, LevelRef out,
                            int level_out, int use_acc, hipStream_t s) {
  const unsigned nb = unsigned(xcd_blocks(total));
#define UB_FWD(TH, TY)                                                                     \
  lks_step_ubatch_kernel<R, TH, TY><<<nb, (NT1<R, TH, TY>), 0, s>>>(d, st, tmap, total, in, \
                                                                    out, level_out, use_acc)
  if (ty == 8) {
    if (thermal) UB_FWD(true, 8);
    else UB_FWD(false, 8);
  } else {
    if (thermal) UB_FWD(true, 4);
    else UB_FWD(false, 4);
  }
#undef UB_FWD
}
template <typename R>
void launch_alks_step_ubatch(const BatchAdj<R>* d, const BatchStore<R>* st, const int* tmap,
                             int total, int ty, bool thermal, int parity, LevelRef lv,
                             int seeded, int b_only, hipStream_t s) {
  const unsigned nb = unsigned(xcd_blocks(total));
#define UB_ADJ(TH, TY)                                                                      \
  alks_step_ubatch_kernel<R, TH, TY><<<nb, (NT1<R, TH, TY>), 0, s>>>(d, st, tmap, total,     \
                                                                     parity, lv, seeded, b_only)
  if (ty == 8) {
    if (thermal) UB_ADJ(true, 8);
    else UB_ADJ(false, 8);
  } else {
    if (thermal) UB_ADJ(true, 4);
    else UB_ADJ(false, 4);
  }
#undef UB_ADJ
}
template <typename R>
void launch_acc_zero_batch(const BatchFwd<R>* d, int nd, hipStream_t s) {
  acc_zero_batch_kernel<R><<<nd, NTHREADS, 0, s>>>(d);
}
template <typename R>
void launch_acc_sum_batch(const BatchFwd<R>* d, int nd, double* out, hipStream_t s) {
  acc_sum_batch_kernel<R><<<nd, NTHREADS, 0, s>>>(d, out);
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
  template void launch_alks_step<R>(const Geo&, const AdjArgs<R>&, hipStream_t);              \
  template void launch_pressure_drop<R>(const Geo&, const uint8_t*, const R*, double*,        \
                                        hipStream_t);                                         \
  template void launch_probe_heat<R>(const Geo&, const uint8_t*, const R*, const R*, double*,  \
                                     hipStream_t);                                            \
  template void launch_source_coef<R>(const Geo&, const double*, double, double, R*, R*,      \
                                      hipStream_t);                                           \
  template void launch_source_heat<R>(const Geo&, const R*, const R*, double*, hipStream_t);  \
  template void launch_probe_T<R>(const Geo&, const uint8_t*, const R*, double*, hipStream_t); \
  template void launch_fill_r<R>(R*, size_t, hipStream_t);                                    \
  template void launch_lks_step_batch<R>(const BatchFwd<R>*, const int*, int, int, bool, int,      \
                                         hipStream_t);                                        \
  template void launch_alks_step_batch<R>(const BatchAdj<R>*, const int*, int, int, bool, int,     \
                                          int, hipStream_t);                                  \
  template void launch_pressure_drop_batch<R>(const BatchFwd<R>*, int, int, double*, hipStream_t); \
  template void launch_lks_step_ubatch<R>(const BatchFwd<R>*, const BatchStore<R>*, const int*,   \
                                          int, int, bool, LevelRef, LevelRef, int, int,        \
                                          hipStream_t);                                        \
  template void launch_alks_step_ubatch<R>(const BatchAdj<R>*, const BatchStore<R>*, const int*,  \
                                           int, int, bool, int, LevelRef, int, int, hipStream_t); \
  template void launch_acc_zero_batch<R>(const BatchFwd<R>*, int, hipStream_t);                \
  template void launch_acc_sum_batch<R>(const BatchFwd<R>*, int, double*, hipStream_t);        \
  template void launch_to_double<R>(const R*, double*, size_t, hipStream_t);                  \
  template void launch_from_double<R>(const double*, R*, size_t, hipStream_t);                \
  template void launch_finite_check<R>(const R*, size_t, int*, hipStream_t);

LKS_INSTANTIATE(float)
LKS_INSTANTIATE(double)

}  // namespace lks
