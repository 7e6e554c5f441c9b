// Device-side definitions shared by the LKS/ALKS kernels and their host
// runtime (gfx950). Lattice: D2Q9 with c0=(0,0) c1=(1,0) c2=(0,1) c3=(-1,0)
// c4=(0,-1) c5=(1,1) c6=(-1,1) c7=(-1,-1) c8=(1,-1) and weights 4/9, 1/9,
// 1/36 (Sec. 2.3); the numbering is the one of the boundary matrices of
// Sec. 2.5.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lks {

// Tile of the 2D kernels: 64 nodes along x (one wavefront) by TY rows, 256
// threads (64 x 4). A remainder of a single column/row is merged into the
// last tile so that every tile is at least 2 nodes wide and tall; the
// one-sided boundary stencils then always find their nodes inside the tile
// plus its halo.
constexpr int TX = 64;
constexpr int NTHREADS = 256;
constexpr int NXCD = 8;  // accelerator complex dies of an MI355X

// Workgroup barrier that orders LDS only. __syncthreads() also waits for every
// outstanding global load and store of the wave, which would drain prefetches
// issued one iteration ahead; data exchanged between the waves of a block goes
// through LDS only, so the fences are limited to the local address space.
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// node-class byte
constexpr int FLOW_INTERIOR = 0, FLOW_VELOCITY = 1, FLOW_PRESSURE = 2, FLOW_CORNER = 3;
constexpr int THERM_DIRICHLET = 1, THERM_FLUX = 2;
constexpr int TAG_J_INLET = 16, TAG_J_OUTLET = 32, TAG_PROBE = 64;

struct Geo {
  int nx, ny, N;
  int periodic, thermal;
  int ntx, nty;     // tiles along x and y
  int ty;           // tile height
  double A;         // eq:A
  double Bf;        // B of the fluid, used on boundary nodes
  double drho_out;  // prescribed outlet density minus 1
  double gbx, gby;  // g beta of the Boussinesq force (0: none)
  double Tref;      // its reference temperature
};

__host__ __device__ inline int tiles_along(int n, int t) {
  int k = (n + t - 1) / t;
  if (k > 1 && n % t == 1) --k;
  return k;
}

// Blocks are handed to the XCDs round-robin; block b runs tile
// (b mod 8) * ceil(T/8) + b / 8 so that each XCD owns a contiguous band of
// tile rows and finds the previous step's data of that band in its own L2.
__host__ __device__ inline int xcd_blocks(int tiles) {
  return NXCD * ((tiles + NXCD - 1) / NXCD);
}

// Least-squares completion operators of a ring orientation (host-built in
// double, Sec. 2.5 / Appendix A). Unknown directions unk[] are those with
// c_i.n > 0 in ascending order; known values are those with c_i.n <= 0.
//   flow (velocity node v=0, pressure node v=1):
//     f_unk[a] = sum_q Lf[v][a][q] f_q + Ls[v][a] s + Lk[v][a] kappa T
//   temperature node: g_unk[a] = sum_q Ld[a][q] g_q
//   zero-flux node with normal velocity u_n:
//     kappa = -(sum_q (ga_q - u_n ge_q) g_q) / (A0 - 2 u_n A1 + u_n^2 A2)
//     g_unk[a] = sum_q Lg0[a][q] g_q - kappa (hc[a] - u_n h1[a])
// The kernels read a copy rounded to their arithmetic type (RingOpT<R>),
// which is what they used to form from the double entries at every use.
template <typename T>
struct RingOpT {
  T Lf[2][3][9];
  T Ls[2][3];
  T Lk[2][3];
  T Ld[3][9];
  T Lg0[3][9];
  T ga[9], ge[9];
  T A0, A1, A2;
  T hc[3], h1[3];
  T uw[3], ucx[3], ucy[3];  // weight and velocity of the unknown directions
  int unk[3];
  int pad;
};
using RingOp = RingOpT<double>;

// element-wise conversion of operator tables (host)
template <typename D, typename S>
inline void conv_op(D& d, const S& s) { d = D(s); }
template <typename D, typename S, size_t N>
inline void conv_op(D (&d)[N], const S (&s)[N]) {
  for (size_t i = 0; i < N; ++i) conv_op(d[i], s[i]);
}
template <typename R>
inline RingOpT<R> ring_op_as(const RingOp& s) {
  RingOpT<R> d{};
  conv_op(d.Lf, s.Lf); conv_op(d.Ls, s.Ls); conv_op(d.Lk, s.Lk); conv_op(d.Ld, s.Ld);
  conv_op(d.Lg0, s.Lg0); conv_op(d.ga, s.ga); conv_op(d.ge, s.ge); conv_op(d.A0, s.A0);
  conv_op(d.A1, s.A1); conv_op(d.A2, s.A2); conv_op(d.hc, s.hc); conv_op(d.h1, s.h1);
  conv_op(d.uw, s.uw); conv_op(d.ucx, s.ucx); conv_op(d.ucy, s.ucy); conv_op(d.unk, s.unk);
  return d;
}

// A pointer read through the constant address space: a load whose address
// is the same in every lane then goes through the scalar unit (read only).
template <typename T>
__device__ inline const __attribute__((address_space(4))) T* as_scalar(const T* p) {
  return (const __attribute__((address_space(4))) T*)p;
}

template <typename R>
struct FwdArgs {
  const uint8_t* mask;
  const R* inv1pa;  // 1 / (1 + alpha_gamma)
  const R* B;       // B_gamma (thermal)
  const R* ubx;
  const R* uby;
  const R* Tb;
  const double* ufac;  // inflow factor per level
  int level_out;       // level written by this step
  int level_mid;       // two-step launches: level written by the first step
  const R* d0;
  const R* ux0;
  const R* uy0;
  const R* T0;
  R* d1;
  R* ux1;
  R* uy1;
  R* T1;
  double* acc;  // per-tile objective accumulator, or nullptr
  int objective;
  const R* beta = nullptr;  // heat-source coefficient beta_gamma, or nullptr
  // two-step launches: where the first step's level is kept (fields left
  // null are not written; all null when the level is not kept)
  R* dm = nullptr;
  R* uxm = nullptr;
  R* uym = nullptr;
  R* Tm = nullptr;
};

template <typename R>
struct AdjArgs {
  const uint8_t* mask;
  const R* inv1pa;
  const R* B;
  const R* dA3;  // 3 alpha'(gamma)
  const R* dB;   // B'(gamma)
  const R* ux;   // state at the destination level n
  const R* uy;
  const R* T;
  const R* r0;   // adjoint equilibrium coefficients at level n+1
  const R* vx0;
  const R* vy0;
  const R* th0;
  R* r1;         // ... at level n
  R* vx1;
  R* vy1;
  R* th1;
  const RingOpT<R>* ops;  // 4 ring orientations: -x, +x, -y, +y
  double* sens;  // dJ/dgamma (double)
  int sens_mode; // 0 none, 1 accumulate, 2 overwrite
  int exact;     // 1: exact discrete adjoint of the Brinkman step
  double seed_dp;
  double seed_heat;
  const R* beta = nullptr;   // heat-source coefficient beta_gamma, or nullptr
  const R* dbeta = nullptr;  // beta'(gamma)
  double seed_src = 0.0;     // weight of the heat-exchange objective
  double seed_bt = 0.0;      // dJ/dT at the heated nodes of the heat-sink objective
  int sens_b_only = 0;       // exact mode, level 0: the conductivity term only
};

// one design of a batch: geometry and the arguments of both ping-pong parities
template <typename R>
struct BatchFwd {
  Geo g;
  FwdArgs<R> a[2];
};
template <typename R>
struct BatchAdj {
  Geo g;
  AdjArgs<R> a[2];
};

// Unsteady batches (checkpointed sweeps of many designs). The designs share
// the horizon N and the checkpoint interval K, so the place of a level is
// the same for all of them: checkpoint n / K when K divides n, else a replay
// slot (the density in the ping-pong buffer of the level's parity) when the
// level lies above the base of the segment being replayed, else the
// ping-pong buffers of its parity.
enum { LVL_CKPT = 0, LVL_SLOT = 1, LVL_PING = 2 };
struct LevelRef {
  int kind, idx, par;
};
// where the levels of one design of an unsteady batch are stored
template <typename R>
struct BatchStore {
  R* C;        // checkpoints: ckf fields of N values each
  R* Seg;      // replay slots: slf fields of N values each (no density)
  R* S[2][4];  // ping-pong buffers: drho, ux, uy, T
  int N, ckf, slf;
  int n_ufac;  // entries of the design's inflow-factor table
};
// field f (drho, ux, uy, T) of the level at r; null for T when the fields
// stored per level stop before it (non-thermal designs). The ping-pong
// buffer is picked with a select, not an index: a runtime index into the
// descriptor would move it to per-lane scratch memory.
template <typename R>
__host__ __device__ inline R* level_field(const BatchStore<R>& s, LevelRef r, int f) {
  if (f >= s.ckf) return nullptr;
  R* const ping = r.par ? s.S[1][f] : s.S[0][f];
  if (r.kind == LVL_CKPT) return s.C + (size_t(r.idx) * s.ckf + f) * size_t(s.N);
  if (r.kind == LVL_SLOT)
    return f == 0 ? ping : s.Seg + (size_t(r.idx) * s.slf + (f - 1)) * size_t(s.N);
  return ping;
}

// host: the four ring operators for a given A and fluid B
void build_ring_ops(double A, double Bf, RingOp ops[4]);

// ---------------------------------------------------------------------------
// D3Q19 (three-dimensional extension)
// ---------------------------------------------------------------------------
// Nodes (i, j, l), k = (l ny + j) nx + i. An axis is periodic when its bit
// of `periodic` is set; a node at an end of a non-periodic axis is a
// boundary node: a face node (one coordinate at an end) or an edge/corner
// node (two or three), which copies density, temperature and adjoint
// moments from (i, j', l'), the node one step inwards along y and z.
struct Geo3 {
  int nx, ny, nz, N;
  int periodic;     // bit 0: x, bit 1: y, bit 2: z
  int thermal;
  int zc, zca;      // z-planes per block: LKS step, ALKS update pass (>= 2)
  int zcf;          // z-planes per block of the fused ALKS step (>= 2)
  int fused;        // ALKS step: 1 fused z-march, 0 pull, face and update passes
  double A;         // eq:A
  double Bf;        // B of the fluid, used on boundary nodes
  double drho_out;  // prescribed outlet density minus 1
};

// Least-squares completion operators of a face orientation o = 2 axis +
// (n = +e_axis), the D3Q19 counterpart of RingOp with five unknowns.
template <typename T>
struct FaceOpT {
  T Lf[2][5][19];
  T Ls[2][5];
  T Lk[2][5];
  T Ld[5][19];
  T Lg0[5][19];
  T ga[19], ge[19];
  T A0, A1, A2;
  T hc[5], h1[5];
  T uw[5], uc[5][3];
  int unk[5];
  int pad[3];
};
using FaceOp3 = FaceOpT<double>;
template <typename R>
inline FaceOpT<R> face_op_as(const FaceOp3& s) {
  FaceOpT<R> d{};
  conv_op(d.Lf, s.Lf); conv_op(d.Ls, s.Ls); conv_op(d.Lk, s.Lk); conv_op(d.Ld, s.Ld);
  conv_op(d.Lg0, s.Lg0); conv_op(d.ga, s.ga); conv_op(d.ge, s.ge); conv_op(d.A0, s.A0);
  conv_op(d.A1, s.A1); conv_op(d.A2, s.A2); conv_op(d.hc, s.hc); conv_op(d.h1, s.h1);
  conv_op(d.uw, s.uw); conv_op(d.uc, s.uc); conv_op(d.unk, s.unk);
  return d;
}
void build_face_ops3(double A, double Bf, FaceOp3 ops[6]);

// fields of the forward state: drho, ux, uy, uz, T
template <typename R>
struct Fwd3Args {
  const uint8_t* mask;
  const R* inv1pa;
  const R* B;
  const R* ub[3];      // prescribed velocity
  const R* Tb;         // prescribed temperature
  const double* ufac;  // inflow factor per level
  int level_out;
  const R* s0[5];      // level n
  R* s1[5];            // level n+1
  const int* copy;     // edge and corner nodes, copied after the step
  int ncopy;
  double* acc;         // per-block objective accumulator, or nullptr
  int objective;
};

// fields of the adjoint coefficients: rho~, Vx, Vy, Vz, Theta
template <typename R>
struct Adj3Args {
  const uint8_t* mask;
  const R* inv1pa;
  const R* B;
  const R* dA3;
  const R* dB;
  const R* u[3];       // state at the destination level n
  const R* T;
  const R* p0[5];      // level n+1
  R* p1[5];            // level n
  R* m;                // moments: rho~, u~ (3), s~ (6), T~, q~ (3); 14 N (10 N without T)
  const FaceOpT<R>* ops;  // -x, +x, -y, +y, -z, +z
  const int* face;     // boundary nodes: faces by orientation, then edges and corners
  int nface;
  double* sens;
  int sens_mode;       // 0 none, 1 accumulate, 2 overwrite
  int exact;           // 1: exact discrete adjoint of the Brinkman step
  double seed_dp;
  double seed_heat;
  int sens_b_only = 0;  // exact mode, level 0: the conductivity term only
};

int blocks3(int N);  // blocks of a node-parallel 3D launch (multiple of 8)
// blocks of the z-marching step kernels, each with one objective accumulator
int zblocks3(const Geo3& g);
// z-planes per block for the device: each kernel's launch fills whole rounds of
// its resident blocks
void zplan3(Geo3& g, int rsz);
// edge and corner nodes in increasing order (out may be null); returns the count
int copy_nodes3(const Geo3& g, int* out);
// boundary nodes of the non-periodic axes (out may be null): the face nodes
// of orientation 0..5 (-x, +x, -y, +y, -z, +z) in increasing order, then the
// edge and corner nodes; returns the count
int face_nodes3(const Geo3& g, int* out);
template <typename R>
void launch_coef3(const Geo3& g, const uint8_t* mask, const double* gamma, double alpha_max,
                  double q_alpha, double Kf, double Ks, double qK, R* inv1pa, R* B, R* dA3,
                  R* dB, hipStream_t s);
template <typename R>
void launch_init3(const Geo3& g, const uint8_t* mask, const R* const ub[3], const R* Tb,
                  double ufac0, R* const st[5], hipStream_t s);
template <typename R>
void launch_lks3_step(const Geo3& g, const Fwd3Args<R>& a, hipStream_t s);
template <typename R>
void launch_alks3_step(const Geo3& g, const Adj3Args<R>& a, hipStream_t s);
// objective over tagged nodes: part holds tag_sum3_parts() partial sums
template <typename R>
void launch_tag_sum3(const Geo3& g, const uint8_t* mask, const R* d, const R* ux, const R* T,
                     int objective, double* part, double* out, hipStream_t s);
int tag_sum3_parts();

// kernel launchers (lks_kernels.hip)
template <typename R>
void launch_coef(const Geo& g, const double* gamma, double alpha_max, double q_alpha,
                 double Kf, double Ks, double q_K, R* inv1pa, R* B, R* dA3, R* dB,
                 hipStream_t s);
// heat-source coefficients beta_gamma and beta'(gamma) (eq:betagamma)
template <typename R>
void launch_source_coef(const Geo& g, const double* gamma, double beta_max, double q_beta,
                        R* beta, R* dbeta, hipStream_t s);
template <typename R>
void launch_init(const Geo& g, const uint8_t* mask, const R* ubx, const R* uby, const R* Tb,
                 double fac0, R* d, R* ux, R* uy, R* T, hipStream_t s);
template <typename R>
void launch_lks_step(const Geo& g, const FwdArgs<R>& a, hipStream_t s);
template <typename R>
void launch_alks_step(const Geo& g, const AdjArgs<R>& a, hipStream_t s);
// two steps per launch, FP32 non-thermal steady sweeps: forward n -> n+2
// (level_mid = n+1, level_out = n+2), adjoint n+2 -> n with the level-n state
void launch_lks_step2(const Geo& g, const FwdArgs<float>& a, hipStream_t s);
// FP64 non-thermal forward, two steps per launch
void launch_lks_step2(const Geo& g, const FwdArgs<double>& a, hipStream_t s);
void launch_alks_step2(const Geo& g, const AdjArgs<float>& a, hipStream_t s);
template <typename R>
void launch_pressure_drop(const Geo& g, const uint8_t* mask, const R* d, double* out,
                          hipStream_t s);
template <typename R>
void launch_probe_heat(const Geo& g, const uint8_t* mask, const R* ux, const R* T, double* out,
                       hipStream_t s);
// heat-sink objective of one level: sum of T over the probe-tagged nodes
template <typename R>
void launch_probe_T(const Geo& g, const uint8_t* mask, const R* T, double* out, hipStream_t s);
// heat-exchange objective of one level: sum of beta (T - 1) over all nodes
template <typename R>
void launch_source_heat(const Geo& g, const R* beta, const R* T, double* out, hipStream_t s);
template <typename R>
void launch_lks_step_batch(const BatchFwd<R>* d, const int* tmap, int total, int ty,
                           bool thermal, int parity, hipStream_t s);
template <typename R>
void launch_alks_step_batch(const BatchAdj<R>* d, const int* tmap, int total, int ty,
                            bool thermal, int parity, int last, hipStream_t s);
template <typename R>
void launch_pressure_drop_batch(const BatchFwd<R>* d, int nd, int parity, double* out,
                                hipStream_t s);
// unsteady batches: one LKS step of every design from level `in` to level
// `out` (= level_out), the objective accumulated per tile when use_acc;
// one ALKS step of every design at the state of level `lv` with the
// descriptors' seeds applied when `seeded` (levels 1..N) and the
// sensitivity accumulated; the per-tile accumulators zeroed and summed per
// design (out[d], the order of launch_sum)
template <typename R>
void launch_lks_step_ubatch(const BatchFwd<R>* d, const BatchStore<R>* st, const int* tmap,
                            int total, int ty, bool thermal, LevelRef in, LevelRef out,
                            int level_out, int use_acc, hipStream_t s);
template <typename R>
void launch_alks_step_ubatch(const BatchAdj<R>* d, const BatchStore<R>* st, const int* tmap,
                             int total, int ty, bool thermal, int parity, LevelRef lv,
                             int seeded, int b_only, hipStream_t s);
template <typename R>
void launch_acc_zero_batch(const BatchFwd<R>* d, int nd, hipStream_t s);
template <typename R>
void launch_acc_sum_batch(const BatchFwd<R>* d, int nd, double* out, hipStream_t s);
void launch_sum(const double* v, int n, double* out, hipStream_t s);
// zero one device flag with a kernel (safe inside a captured graph;
// lks_runtime.hip)
void launch_clear_flag(int* flag, hipStream_t s);
void launch_fill(double* p, size_t n, double v, hipStream_t s);
template <typename R>
void launch_fill_r(R* p, size_t n, hipStream_t s);
template <typename R>
void launch_to_double(const R* src, double* dst, size_t n, hipStream_t s);
template <typename R>
void launch_from_double(const double* src, R* dst, size_t n, hipStream_t s);
template <typename R>
void launch_finite_check(const R* a, size_t n, int* flag, hipStream_t s);

}  // namespace lks
