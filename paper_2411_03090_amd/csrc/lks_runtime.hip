// Host runtime and C ABI of the LKS/ALKS library (see include/lks.h).
//
// Owns the problem description, validates it, plans the device workspace
// (state, adjoint, design coefficients, boundary data and -- for unsteady
// problems -- checkpoints every K levels plus one replay segment), and drives
// the forward sweep, the adjoint sweep and the checkpoint replay on one HIP
// stream.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/lks.h"
#include "lks_device.h"

using lks::Geo;

namespace lks {
__global__ void clear_flag_kernel(int* flag) {
  if (threadIdx.x == 0) *flag = 0;
}
void launch_clear_flag(int* flag, hipStream_t s) { clear_flag_kernel<<<1, 64, 0, s>>>(flag); }
}  // namespace lks

namespace {

thread_local std::string g_create_error;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// message of a call on a context without a usable workspace
template <typename C>
const char* unbound_reason(const C* c) {
  return c->static_dev >= 0
             ? "the static workspace was bound by another context since (bind again)"
             : "no workspace bound";
}

// One action of a binomial reversal schedule: advance `steps` LKS steps from
// the level `from` held in snapshot `src` (the last step writes snapshot
// `dst`, or the working buffers when dst < 0), or run the ALKS step of level
// `from` with its state in snapshot `src` (src < 0: the working buffers).
struct Act {
  int adjoint;
  int from, steps, src, dst;
};

struct Plan {
  int scheme = 0;     // LKS_CKPT_TWO_LEVEL or LKS_CKPT_BINOMIAL (unsteady)
  int K = 0;          // two-level: checkpoint interval (N+1: whole trajectory kept)
  int n_ckpt = 0;     // two-level: checkpoints at levels 0, K, 2K, ..., ls;
                      // binomial: snapshots (level 0 and s free slots)
  int n_slots = 0;    // replay segment slots (K-1)
  int ls = 0;         // level of the last checkpoint
  long long replay = 0;  // LKS steps the adjoint sweep recomputes
  size_t ckpt_bytes = 0;
  size_t total = 0;
  std::vector<Act> acts;  // binomial: forward placements, then the reversal
  int n_pre = 0;          // binomial: leading actions done by the forward pass
};

}  // namespace

struct lks_ctx {
  lks_grid grid{};
  lks_phys phys{};
  int objective = 0, mode = 0, n_steps = 0;
  double rho_out = 1.0;
  std::vector<uint8_t> mask;
  std::vector<double> ubar, Tbar, ufac;
  int n_in = 0, n_out = 0, n_probe = 0;
  int dim = 2;         // 2: D2Q9, 3: D3Q19
  int spl_f = 1;       // steady sweeps: time steps per launch (1 or 2),
  int spl_a = 1;       // forward and adjoint
  int N = 0;           // nodes
  Geo geo{};           // D2Q9 geometry
  lks::Geo3 geo3{};    // D3Q19 geometry
  hipStream_t stream = nullptr;
  size_t budget = 0;
  int rsz = 8;
  Plan plan;
  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool bound = false;
  int static_dev = -1;    // device whose static scratch array is bound, or -1
  // mixed precision: the FP32 context that runs the adjoint sweep (this
  // context runs the forward sweep in FP64)
  lks_ctx* lo = nullptr;
  // carved device pointers (element type depends on precision)
  uint8_t* d_mask = nullptr;
  void *ubx = nullptr, *uby = nullptr, *ubz = nullptr, *Tb = nullptr;
  double* d_ufac = nullptr;
  void *inv1pa = nullptr, *B = nullptr, *dA3 = nullptr, *dB = nullptr;
  void *beta = nullptr, *dbeta = nullptr;  // heat source (beta_max > 0)
  // forward ping-pong: drho, ux, uy, T (D2Q9) or drho, ux, uy, uz, T (D3Q19)
  void* S[2][5] = {};
  // adjoint ping-pong: rho~, Vx, Vy, Theta or rho~, Vx, Vy, Vz, Theta
  void* P[2][5] = {};
  void* C = nullptr;     // checkpoints
  void* Seg = nullptr;   // replay segment
  void* d_ops = nullptr;   // adjoint boundary operators (4 orientations), RingOpT<R>
  lks::RingOp ops[4];
  lks::RingOpT<float> ops_f[4];
  void* d_ops3 = nullptr;  // D3Q19 face operators (6 orientations), FaceOpT<R>
  lks::FaceOp3 ops3[6];
  lks::FaceOpT<float> ops3_f[6];
  int* copy3 = nullptr;  // D3Q19 edge and corner nodes (device)
  int* face3 = nullptr;  // D3Q19 boundary nodes by orientation (device)
  void* M3 = nullptr;    // D3Q19 adjoint moments of one step
  std::vector<int> copy3h, face3h;
  double* acc = nullptr; // per-tile objective accumulators
  double* scal = nullptr;
  int* flag = nullptr;
  // run state
  bool have_forward = false;
  bool have_adjoint = false;
  int adj_exact = 0;     // LKS_ADJ_EXACT: transpose of the discrete Brinkman step
  int ckpt_scheme = 0;   // requested checkpointing (LKS_CKPT_*)
  int ckpt_slots = 0;    // binomial: requested free snapshot slots (0: budget)
  void* lastv[5] = {};   // unsteady: where the last forward level is held
  int cur = 0;      // steady forward: ping-pong index of the current level
  int acur = 0;     // adjoint: ping-pong index of the current level
  int last_level = 0;
  std::string err;
};

namespace {

lks_status fail(lks_ctx* c, lks_status s, const std::string& msg) {
  if (c) c->err = msg;
  else g_create_error = msg;
  return s;
}

bool hip_ok(lks_ctx* c, hipError_t e, const char* what, lks_status* st) {
  if (e == hipSuccess) return true;
  *st = fail(c, LKS_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return false;
}

int n_tiles(const Geo& g) { return g.ntx * g.nty; }
// tiles of the smallest tile height the kernels support (sizes accumulators)
int max_tiles(const Geo& g) {
  return lks::tiles_along(g.nx, lks::TX) * lks::tiles_along(g.ny, 4);
}
constexpr int TILE_ROWS[3] = {4, 8, 16};
// 64 x 16 tiles exist for FP32 non-thermal D2Q9 problems only (LDS size)
bool tile_rows_ok(int ty, int rsz, int thermal) {
  return ty == 4 || ty == 8 || (ty == 16 && rsz == 4 && !thermal);
}
void set_tile_rows(Geo& g, int ty) {
  g.ty = ty;
  g.ntx = lks::tiles_along(g.nx, lks::TX);
  g.nty = lks::tiles_along(g.ny, ty);
}

// state fields per level (the last one is T) and the stored ones
int nfields(const lks_ctx* c) { return c->dim == 3 ? 5 : 4; }
int tfield(const lks_ctx* c) { return nfields(c) - 1; }
// fields stored per checkpoint / per replay slot (the replay keeps drho in
// the ping-pong buffers)
int ckpt_fields(const lks_ctx* c) { return c->phys.thermal ? nfields(c) : nfields(c) - 1; }
int slot_fields(const lks_ctx* c) { return ckpt_fields(c) - 1; }
// per-block objective accumulators of an unsteady forward sweep
int acc_count(const lks_ctx* c) {
  return c->dim == 3 ? lks::zblocks3(c->geo3) : n_tiles(c->geo);
}
int acc_bound3(const lks_ctx* c) {
  const lks::Geo3& g = c->geo3;
  return ((g.nx + 63) / 64) * ((g.ny + 3) / 4) * std::max(1, g.nz / 2);
}
// D3Q19 adjoint moments between the two passes of a step: 14, 10 without T
int moments3_fields(const lks_ctx* c) { return c->phys.thermal ? 14 : 10; }
// (D3Q19 steady runs also take the partial sums of the objective there)
int acc_capacity(const lks_ctx* c) {
  return c->dim == 3 ? std::max(acc_bound3(c), lks::tag_sum3_parts()) : max_tiles(c->geo);
}

size_t traj_bytes(const lks_ctx* c, int K) {
  const size_t N = size_t(c->N), r = size_t(c->rsz);
  const int n = c->n_steps;
  size_t n_ckpt = size_t(n / K) + 1;
  return n_ckpt * ckpt_fields(c) * N * r + size_t(K - 1) * slot_fields(c) * N * r;
}

bool has_source(const lks_ctx* c) { return c->phys.beta_max > 0.0; }

size_t base_bytes(const lks_ctx* c) {
  const size_t N = size_t(c->N), r = size_t(c->rsz);
  const int nf = nfields(c);
  size_t b = 0;
  b += align256(N);                          // mask
  b += size_t(c->dim + 1) * align256(N * r);  // prescribed velocity, T
  b += align256(sizeof(double) * c->ufac.size());
  b += (has_source(c) ? 6 : 4) * align256(N * r);  // coefficients
  b += 2 * nf * align256(N * r);             // forward ping-pong
  b += 2 * nf * align256(N * r);             // adjoint ping-pong
  b += align256(sizeof(double) * acc_capacity(c));
  if (c->dim == 3) {
    b += align256(6 * sizeof(lks::FaceOp3));  // face operators
    b += align256(sizeof(int) * c->copy3h.size());  // edge and corner nodes
    b += align256(sizeof(int) * c->face3h.size());  // boundary nodes
    b += align256(size_t(moments3_fields(c)) * N * r);
  } else {
    b += align256(4 * sizeof(lks::RingOp));   // ring operators
  }
  b += align256(sizeof(double) * 8);
  b += align256(sizeof(int) * 4);
  return b;
}

// ---- binomial checkpointing (Griewank's reversal schedule) ----------------
// beta(c, r) = C(c + r, c): the most levels that c snapshots can reverse when
// no step is evaluated more than r times (saturates at 2^62).
long long beta_cr(int c, int r) {
  if (r < 0 || c < 0) return 0;
  long long b = 1;
  const int k = std::min(c, r);
  for (int i = 1; i <= k; ++i) {
    const long long num = (long long)(c + r - k + i);
    if (b > (1LL << 62) / num) return 1LL << 62;
    b = b * num / i;
  }
  return b;
}

// Steps to advance before the next snapshot when levels a..a+t are to be
// reversed with the level a in a snapshot and s free slots: with l = t + 1
// levels, c = s + 1 snapshots and r the least repetition count with
// beta(c, r) >= l, k = min(t - beta(c - 1, r - 1) + 1, beta(c, r - 1)),
// which attains the least number of recomputed steps.
int binomial_split(int t, int s) {
  const long long l = (long long)t + 1;
  const int c = s + 1;
  int r = 0;
  while (beta_cr(c, r) < l) ++r;
  long long k = std::min((long long)t - beta_cr(c - 1, r - 1) + 1, beta_cr(c, r - 1));
  return int(std::max(1LL, std::min((long long)t, k)));
}

// Appends the reversal of levels a..b (level a in snapshot sa; `free_` lists
// the free snapshots, lowest first) to acts.
void binomial_reverse(std::vector<Act>& acts, int a, int b, int sa, std::vector<int>& free_) {
  while (true) {
    if (a == b) {
      acts.push_back({1, a, 0, sa, -1});
      return;
    }
    if (free_.empty()) {
      for (int n = b; n > a; --n) {
        acts.push_back({0, a, n - a, sa, -1});
        acts.push_back({1, n, 0, -1, -1});
      }
      acts.push_back({1, a, 0, sa, -1});
      return;
    }
    const int m = a + binomial_split(b - a, int(free_.size()));
    const int j = free_.front();
    free_.erase(free_.begin());
    acts.push_back({0, a, m - a, sa, j});
    binomial_reverse(acts, m, b, j, free_);
    free_.insert(std::lower_bound(free_.begin(), free_.end(), j), j);
    b = m - 1;  // then levels a..m-1 with the same snapshots
  }
}

// Schedule for n steps with s free snapshots: acts holds the whole reversal;
// its leading advances into snapshots (the first descent) are the ones the
// forward sweep performs on its way to level n.
void binomial_plan(Plan& p, int n, int s) {
  p.acts.clear();
  std::vector<int> free_;
  for (int j = 1; j <= s; ++j) free_.push_back(j);
  binomial_reverse(p.acts, 0, n, 0, free_);
  p.n_pre = 0;
  while (p.n_pre < int(p.acts.size()) && !p.acts[p.n_pre].adjoint && p.acts[p.n_pre].dst >= 0)
    ++p.n_pre;
  p.replay = 0;
  for (size_t i = size_t(p.n_pre); i < p.acts.size(); ++i)
    if (!p.acts[i].adjoint) p.replay += p.acts[i].steps;
}

size_t snapshot_bytes(const lks_ctx* c) {
  return size_t(ckpt_fields(c)) * size_t(c->N) * size_t(c->rsz);
}

lks_status plan_binomial(lks_ctx* c, Plan& p, size_t base) {
  const int n = c->n_steps;
  const size_t one = snapshot_bytes(c);
  int s = c->ckpt_slots;
  if (s == 0) {
    // as many free snapshots as the budget holds, at most one per level
    if (c->budget == 0) {
      s = n;
    } else {
      if (c->budget < base + one) return fail(nullptr, LKS_E_NOMEM,
          "memory budget below one snapshot of the state");
      s = int(std::min<size_t>((c->budget - base) / one - 1, size_t(n)));
      while (s > 0 && base + align256(size_t(s + 1) * one) > c->budget) --s;
    }
  }
  s = std::min(s, n);
  const size_t need = base + align256(size_t(s + 1) * one);
  if (c->budget != 0 && need > c->budget) {
    char buf[160];
    snprintf(buf, sizeof buf, "memory budget %zu B below the %d-snapshot plan (%zu B)",
             c->budget, s, need);
    return fail(nullptr, LKS_E_NOMEM, buf);
  }
  p.scheme = LKS_CKPT_BINOMIAL;
  p.n_ckpt = s + 1;
  p.n_slots = 0;
  p.K = 0;
  p.ls = 0;
  p.ckpt_bytes = size_t(s + 1) * one;
  p.total = need;
  binomial_plan(p, n, s);
  return LKS_OK;
}

// Unsteady problems: two-level checkpointing unless binomial checkpointing
// is requested, or no two-level plan fits the budget and the scheme is
// automatic. Among the intervals K whose storage fits the budget, the plan
// takes the one that replays the fewest forward steps (ls - ls/K with
// ls = (N/K) K, which grows with K; K = N+1 keeps every level and replays
// none), and of equal replay counts the one that needs the least memory.
// Checkpoint and segment levels are written by the step kernels in place,
// so a smaller interval costs no extra copies in the forward sweep.
// the two-level plan with checkpoint interval K
void set_two_level(lks_ctx* c, int K) {
  const int n = c->n_steps;
  Plan p;
  p.K = K;
  p.n_ckpt = n / K + 1;
  p.n_slots = K - 1;
  p.ls = (n / K) * K;
  p.ckpt_bytes = traj_bytes(c, K);
  p.total = base_bytes(c) + align256(size_t(p.n_ckpt) * ckpt_fields(c) * c->N * c->rsz) +
            align256(size_t(p.n_slots) * slot_fields(c) * c->N * c->rsz);
  p.scheme = LKS_CKPT_TWO_LEVEL;
  p.replay = K > n ? 0 : (long long)p.ls - (long long)p.ls / K;
  c->plan = std::move(p);
}

lks_status plan_memory(lks_ctx* c) {
  Plan p;
  size_t base = base_bytes(c);
  if (c->mode != LKS_UNSTEADY) {
    p.total = base;
    c->plan = p;
    return LKS_OK;
  }
  if (c->ckpt_scheme == LKS_CKPT_BINOMIAL) {
    lks_status st = plan_binomial(c, p, base);
    if (st == LKS_OK) c->plan = std::move(p);
    return st;
  }
  const int n = c->n_steps;
  int best = 0;
  long long best_rep = 0;
  size_t best_t = 0;
  for (int K = 1; K <= n + 1; ++K) {
    const size_t t = traj_bytes(c, K) + 2 * 256;
    if (c->budget != 0 && base + t > c->budget) continue;
    const long long ls = (long long)(n / K) * K;
    const long long rep = K > n ? 0 : ls - ls / K;
    if (best == 0 || rep < best_rep || (rep == best_rep && t < best_t)) {
      best = K;
      best_rep = rep;
      best_t = t;
    }
  }
  if (best == 0 && c->ckpt_scheme == LKS_CKPT_AUTO) {
    lks_status st = plan_binomial(c, p, base);
    if (st == LKS_OK) c->plan = std::move(p);
    return st;
  }
  if (best == 0) {
    // report the smallest footprint for the message
    size_t mn = ~size_t(0);
    for (int K = 1; K <= n + 1; ++K) mn = std::min(mn, traj_bytes(c, K));
    char buf[160];
    snprintf(buf, sizeof buf, "memory budget %zu B below the smallest checkpoint plan (%zu B)",
             c->budget, base + mn);
    return fail(nullptr, LKS_E_NOMEM, buf);
  }
  set_two_level(c, best);
  return LKS_OK;
}

// checks shared by both lattices
lks_status validate_common(const lks_grid* gr, const lks_phys* ph, const lks_bc* bc) {
  if (gr->precision != LKS_FP64 && gr->precision != LKS_FP32DEV)
    return fail(nullptr, LKS_E_INVALID, "unknown precision");
  if (!(ph->nu > 0.0 && ph->nu < 1.0 / 6.0))
    return fail(nullptr, LKS_E_INVALID, "nu must lie in (0, 1/6) (A > 0, eq:A)");
  if (!(ph->alpha_max >= 0.0) || !(ph->q_alpha > 0.0))
    return fail(nullptr, LKS_E_INVALID, "alpha_max must be >= 0 and q_alpha > 0");
  if (ph->thermal) {
    if (!(ph->Pr > 0.0) || !(ph->Ks_over_Kf >= 0.0) || !(ph->q_K > 0.0))
      return fail(nullptr, LKS_E_INVALID, "Pr, q_K must be > 0 and Ks/Kf >= 0");
    double Kf = ph->nu / ph->Pr, Ks = Kf * ph->Ks_over_Kf;
    if (Kf > 1.0 / 6.0 || Ks > 1.0 / 6.0)
      return fail(nullptr, LKS_E_INVALID, "diffusivity above 1/6 gives B < 0 (eq:B)");
  }
  if (!bc->node_class || !bc->u_bar) return fail(nullptr, LKS_E_INVALID, "null boundary data");
  if (ph->thermal && !bc->T_bar) return fail(nullptr, LKS_E_INVALID, "thermal needs T_bar");
  const bool force = ph->gbeta[0] != 0.0 || ph->gbeta[1] != 0.0 || ph->gbeta[2] != 0.0;
  if (!std::isfinite(ph->gbeta[0]) || !std::isfinite(ph->gbeta[1]) ||
      !std::isfinite(ph->gbeta[2]) || !std::isfinite(ph->T_ref))
    return fail(nullptr, LKS_E_INVALID, "Boussinesq parameters not finite");
  if (force && !ph->thermal)
    return fail(nullptr, LKS_E_INVALID, "the Boussinesq force needs a thermal problem");
  if (force && gr->lattice == LKS_D3Q19)
    return fail(nullptr, LKS_E_UNSUPPORTED, "the Boussinesq force is D2Q9 only");
  if (!std::isfinite(ph->beta_max) || !(ph->beta_max >= 0.0))
    return fail(nullptr, LKS_E_INVALID, "beta_max must be finite and >= 0");
  const bool source = ph->beta_max > 0.0;
  if (source && !(ph->q_beta > 0.0 && std::isfinite(ph->q_beta)))
    return fail(nullptr, LKS_E_INVALID, "the heat source needs q_beta > 0");
  if (source && !ph->thermal)
    return fail(nullptr, LKS_E_INVALID, "the heat source needs a thermal problem");
  if (source && gr->lattice == LKS_D3Q19)
    return fail(nullptr, LKS_E_UNSUPPORTED, "the heat source is D2Q9 only");
  if (bc->objective != LKS_OBJ_PRESSURE_DROP && bc->objective != LKS_OBJ_HEAT &&
      bc->objective != LKS_OBJ_HEAT_EXCHANGE && bc->objective != LKS_OBJ_HEAT_SINK)
    return fail(nullptr, LKS_E_INVALID, "unknown objective");
  if (bc->objective == LKS_OBJ_HEAT_SINK && !ph->thermal)
    return fail(nullptr, LKS_E_INVALID, "the heat-sink objective needs a thermal problem");
  if (bc->objective == LKS_OBJ_HEAT_SINK && gr->lattice == LKS_D3Q19)
    return fail(nullptr, LKS_E_UNSUPPORTED, "the heat-sink objective is D2Q9 only");
  if (ph->thermal)
    for (long long k = 0; k < (long long)gr->nx * gr->ny * std::max(gr->nz, 1); ++k)
      if (!std::isfinite(bc->T_bar[k])) return fail(nullptr, LKS_E_INVALID, "T_bar not finite");
  if (bc->objective == LKS_OBJ_HEAT_EXCHANGE && !source)
    return fail(nullptr, LKS_E_INVALID, "the heat-exchange objective needs the heat source");
  if (bc->objective == LKS_OBJ_HEAT && !ph->thermal)
    return fail(nullptr, LKS_E_INVALID, "heat objective needs a thermal problem");
  if (bc->mode != LKS_STEADY && bc->mode != LKS_UNSTEADY)
    return fail(nullptr, LKS_E_INVALID, "unknown mode");
  if (bc->mode == LKS_UNSTEADY && bc->n_steps < 1)
    return fail(nullptr, LKS_E_INVALID, "unsteady needs n_steps >= 1");
  if (bc->u_factor && bc->n_factor < 1) return fail(nullptr, LKS_E_INVALID, "n_factor < 1");
  if (!(bc->rho_out > 0.0)) return fail(nullptr, LKS_E_INVALID, "rho_out must be > 0");
  if (bc->u_factor)
    for (int n = 0; n < bc->n_factor; ++n)
      if (!std::isfinite(bc->u_factor[n])) return fail(nullptr, LKS_E_INVALID, "u_factor not finite");
  return LKS_OK;
}

double factor_max(const lks_bc* bc) {
  double fmax = 1.0;
  if (bc->u_factor)
    for (int n = 0; n < bc->n_factor; ++n) fmax = std::max(fmax, std::fabs(bc->u_factor[n]));
  return fmax;
}

lks_status validate(const lks_grid* gr, const lks_phys* ph, const lks_bc* bc) {
  if (!gr || !ph || !bc) return fail(nullptr, LKS_E_INVALID, "null descriptor");
  if (gr->lattice != LKS_D2Q9) return fail(nullptr, LKS_E_INVALID, "unknown lattice");
  if (gr->nz > 1) return fail(nullptr, LKS_E_INVALID, "nz must be 1 for D2Q9");
  const int minn = gr->periodic ? 3 : 4;
  if (gr->nx < minn || gr->ny < minn) return fail(nullptr, LKS_E_INVALID, "grid too small");
  if ((long long)gr->nx * gr->ny > (1LL << 31) / 16)
    return fail(nullptr, LKS_E_INVALID, "grid too large");
  lks_status st = validate_common(gr, ph, bc);
  if (st != LKS_OK) return st;
  const int nx = gr->nx, ny = gr->ny, N = nx * ny;
  double fmax = 1.0;
  if (bc->u_factor)
    for (int n = 0; n < bc->n_factor; ++n) {
      if (!std::isfinite(bc->u_factor[n])) return fail(nullptr, LKS_E_INVALID, "u_factor not finite");
      fmax = std::max(fmax, std::fabs(bc->u_factor[n]));
    }
  for (int k = 0; k < N; ++k) {
    const int i = k % nx, j = k / nx;
    const int m = bc->node_class[k];
    if (m & 0x80) return fail(nullptr, LKS_E_INVALID, "reserved node-class bit set");
    const double u = std::hypot(bc->u_bar[k], bc->u_bar[N + k]) * fmax;
    if (!(u <= 0.3)) return fail(nullptr, LKS_E_INVALID, "prescribed |u| above 0.3");
    if (gr->periodic) continue;
    const bool ring = i == 0 || j == 0 || i == nx - 1 || j == ny - 1;
    const bool corner = (i == 0 || i == nx - 1) && (j == 0 || j == ny - 1);
    const int fc = m & 3, tc = (m >> 2) & 3;
    if (corner) {
      if (fc != LKS_FLOW_CORNER) return fail(nullptr, LKS_E_INVALID, "corner node not classed corner");
      if (m & (LKS_TAG_J_INLET | LKS_TAG_J_OUTLET | LKS_TAG_PROBE))
        return fail(nullptr, LKS_E_INVALID, "corner nodes carry no objective tag");
    } else if (ring) {
      if (fc != LKS_FLOW_VELOCITY && fc != LKS_FLOW_PRESSURE)
        return fail(nullptr, LKS_E_INVALID, "ring node needs a velocity or pressure class");
      if (bc->objective == LKS_OBJ_HEAT_SINK && (m & LKS_TAG_PROBE) && tc != 2)
        return fail(nullptr, LKS_E_INVALID, "heated boundary nodes need the heat-flux class");
      if (ph->thermal && tc != 1 && tc != 2)
        return fail(nullptr, LKS_E_INVALID, "ring node needs a thermal class");
    } else {
      if (fc != LKS_FLOW_INTERIOR || tc != 0)
        return fail(nullptr, LKS_E_INVALID, "interior node with a boundary class");
      if (m & (LKS_TAG_J_INLET | LKS_TAG_J_OUTLET))
        return fail(nullptr, LKS_E_INVALID, "pressure-drop tags belong on ring nodes");
      if (bc->objective == LKS_OBJ_HEAT_SINK && (m & LKS_TAG_PROBE))
        return fail(nullptr, LKS_E_INVALID, "the heated boundary lies on ring nodes");
    }
    if (tc == 3) return fail(nullptr, LKS_E_INVALID, "unknown thermal class");
  }
  if (bc->objective == LKS_OBJ_HEAT_SINK) {
    if (gr->periodic) return fail(nullptr, LKS_E_INVALID, "the heat-sink objective needs a boundary");
    int heated = 0;
    for (int k = 0; k < N; ++k) heated += (bc->node_class[k] & LKS_TAG_PROBE) ? 1 : 0;
    if (!heated) return fail(nullptr, LKS_E_INVALID, "the heat-sink objective needs heated nodes");
  }
  return LKS_OK;
}

// D3Q19: grid->periodic is a bit mask of periodic axes (bit 0 x, bit 1 y,
// bit 2 z). Face nodes (one coordinate at an end of a non-periodic axis)
// need a velocity or pressure class (and a thermal class); edge and corner
// nodes the copy class and no tag; interior nodes the interior class, with
// an optional prescribed temperature (a solid held at T_bar) and the SOLID
// tag for non-design nodes.
lks_status validate3(const lks_grid* gr, const lks_phys* ph, const lks_bc* bc) {
  if (gr->periodic < 0 || gr->periodic > 7)
    return fail(nullptr, LKS_E_INVALID, "periodic must be an axis mask 0..7 for D3Q19");
  const int n3[3] = {gr->nx, gr->ny, gr->nz};
  for (int a = 0; a < 3; ++a)
    if (n3[a] < (((gr->periodic >> a) & 1) ? 3 : 4))
      return fail(nullptr, LKS_E_INVALID, "grid too small");
  if ((long long)gr->nx * gr->ny * gr->nz > (1LL << 31) / 16)
    return fail(nullptr, LKS_E_INVALID, "grid too large");
  lks_status st = validate_common(gr, ph, bc);
  if (st != LKS_OK) return st;
  const long long N = (long long)gr->nx * gr->ny * gr->nz;
  const double fmax = factor_max(bc);
  for (long long k = 0; k < N; ++k) {
    const int x[3] = {int(k % gr->nx), int((k / gr->nx) % gr->ny), int(k / ((long long)gr->nx * gr->ny))};
    int ne = 0;
    for (int a = 0; a < 3; ++a)
      if (!((gr->periodic >> a) & 1) && (x[a] == 0 || x[a] == n3[a] - 1)) ++ne;
    const int m = bc->node_class[k];
    const double u = std::sqrt(bc->u_bar[k] * bc->u_bar[k] + bc->u_bar[N + k] * bc->u_bar[N + k] +
                               bc->u_bar[2 * N + k] * bc->u_bar[2 * N + k]) * fmax;
    if (!(u <= 0.3)) return fail(nullptr, LKS_E_INVALID, "prescribed |u| above 0.3");
    const int fc = m & 3, tc = (m >> 2) & 3;
    if (tc == 3) return fail(nullptr, LKS_E_INVALID, "unknown thermal class");
    if (ne >= 2) {
      if (fc != LKS_FLOW_CORNER) return fail(nullptr, LKS_E_INVALID, "edge node not classed copy");
      if (m & (LKS_TAG_J_INLET | LKS_TAG_J_OUTLET | LKS_TAG_PROBE | LKS_TAG_SOLID))
        return fail(nullptr, LKS_E_INVALID, "edge nodes carry no tag");
    } else if (ne == 1) {
      if (fc != LKS_FLOW_VELOCITY && fc != LKS_FLOW_PRESSURE)
        return fail(nullptr, LKS_E_INVALID, "face node needs a velocity or pressure class");
      if (ph->thermal && tc != 1 && tc != 2)
        return fail(nullptr, LKS_E_INVALID, "face node needs a thermal class");
      if (m & LKS_TAG_SOLID) return fail(nullptr, LKS_E_INVALID, "SOLID tags interior nodes");
    } else {
      if (fc != LKS_FLOW_INTERIOR || tc == 2)
        return fail(nullptr, LKS_E_INVALID, "interior node with a boundary class");
      if (tc == 1 && !ph->thermal)
        return fail(nullptr, LKS_E_INVALID, "prescribed temperature needs a thermal problem");
      if (m & (LKS_TAG_J_INLET | LKS_TAG_J_OUTLET))
        return fail(nullptr, LKS_E_INVALID, "pressure-drop tags belong on face nodes");
    }
  }
  return LKS_OK;
}

template <typename R>
R* rp(void* p) { return static_cast<R*>(p); }

// ---------------------------------------------------------------------------
// drivers
// ---------------------------------------------------------------------------
template <typename R>
struct Run {
  lks_ctx* c;
  const Geo& g;
  size_t N;
  int nf;  // state fields per level; the last is T
  explicit Run(lks_ctx* cc) : c(cc), g(cc->geo), N(size_t(cc->N)), nf(nfields(cc)) {}

  R* ckpt(int m, int f) { return rp<R>(c->C) + (size_t(m) * ckpt_fields(c) + f) * N; }
  R* slot(int s, int f) { return rp<R>(c->Seg) + (size_t(s) * slot_fields(c) + f) * N; }
  R* cur_field(int f) { return rp<R>(c->S[c->cur][f]); }

  // pointers (drho, u..., T) of level n of an unsteady run; seg_base is the
  // first level of the segment held in the replay slots; T is null when the
  // problem is not thermal. What a checkpoint or slot does not hold (drho of
  // a slot level, every field of a level between checkpoints) lives in the
  // ping-pong buffers pp (n & 1 unless the sweep tracks it: the adjoint reads
  // only u and T, which never live there).
  void level(int n, int seg_base, R* out[5], int pp = -1) {
    const int K = c->plan.K, nst = ckpt_fields(c);
    if (pp < 0) pp = n & 1;
    for (int f = 0; f < 5; ++f) out[f] = nullptr;
    if (n % K == 0) {
      const int m = n / K;
      for (int f = 0; f < nst; ++f) out[f] = ckpt(m, f);
      return;
    }
    if (n > seg_base) {
      const int s = n - seg_base - 1;
      out[0] = rp<R>(c->S[pp][0]);
      for (int f = 1; f < nst; ++f) out[f] = slot(s, f - 1);
      return;
    }
    for (int f = 0; f < nf; ++f) out[f] = rp<R>(c->S[pp][f]);
    if (!c->phys.thermal) out[nf - 1] = nullptr;
  }

  // LKS steps from level `from` to level `to` of an unsteady two-level plan,
  // each level where level() puts it for seg_base, the objective into acc
  // when given. With two steps per launch a launch skips the level between
  // (or writes what a checkpoint or slot keeps of it), so the ping-pong
  // buffer is tracked here rather than taken from the level's parity; the
  // pointers of level `to` are returned in last.
  void sweep(int from, int to, int seg_base, double* acc, R* last[5]) {
    const bool two = c->dim == 2 && two_step_fwd(c->spl_f);
    int pp = 0;  // the ping-pong buffers of the current level
    R* in[5];
    level(from, seg_base, in, pp);
    for (int n = from; n < to;) {
      R* out[5];
      if (two && n + 2 <= to) {
        R* mid[5];
        level(n + 1, seg_base, mid, pp ^ 1);
        level(n + 2, seg_base, out, pp ^ 1);
        // what of the middle level is kept: the checkpoint or slot fields
        for (int f = 0; f < 5; ++f)
          if (mid[f] && (mid[f] == rp<R>(c->S[0][f]) || mid[f] == rp<R>(c->S[1][f])))
            mid[f] = nullptr;
        lks::FwdArgs<R> a = fwd_args(in, out, n + 2, acc);
        a.dm = mid[0];
        a.uxm = mid[1];
        a.uym = mid[2];
        a.Tm = mid[3];
        lks::launch_lks_step2(g, a, c->stream);
        n += 2;
      } else {
        level(n + 1, seg_base, out, pp ^ 1);
        step(in, out, n + 1, acc);
        n += 1;
      }
      pp ^= 1;
      for (int f = 0; f < 5; ++f) in[f] = out[f];
    }
    for (int f = 0; f < 5; ++f) last[f] = in[f];
  }

  void step(R* const in[5], R* const out[5], int level_out, double* acc) {
    if (c->dim == 3) {
      lks::Fwd3Args<R> a;
      a.mask = c->d_mask;
      a.inv1pa = rp<R>(c->inv1pa);
      a.B = rp<R>(c->B);
      a.ub[0] = rp<R>(c->ubx);
      a.ub[1] = rp<R>(c->uby);
      a.ub[2] = rp<R>(c->ubz);
      a.Tb = rp<R>(c->Tb);
      a.ufac = c->d_ufac;
      a.level_out = std::min(level_out, int(c->ufac.size()) - 1);
      for (int f = 0; f < 5; ++f) {
        a.s0[f] = in[f];
        a.s1[f] = out[f];
      }
      a.copy = c->copy3;
      a.ncopy = int(c->copy3h.size());
      a.acc = acc;
      a.objective = c->objective;
      lks::launch_lks3_step<R>(c->geo3, a, c->stream);
      return;
    }
    lks::launch_lks_step<R>(g, fwd_args(in, out, level_out, acc), c->stream);
  }

  lks::FwdArgs<R> fwd_args(R* const in[5], R* const out[5], int level_out, double* acc) {
    lks::FwdArgs<R> a;
    a.mask = c->d_mask;
    a.inv1pa = rp<R>(c->inv1pa);
    a.B = rp<R>(c->B);
    a.ubx = rp<R>(c->ubx);
    a.uby = rp<R>(c->uby);
    a.Tb = rp<R>(c->Tb);
    a.ufac = c->d_ufac;
    a.level_out = std::min(level_out, int(c->ufac.size()) - 1);
    a.level_mid = std::min(std::max(level_out - 1, 0), int(c->ufac.size()) - 1);
    a.d0 = in[0];
    a.ux0 = in[1];
    a.uy0 = in[2];
    a.T0 = in[3];
    a.d1 = out[0];
    a.ux1 = out[1];
    a.uy1 = out[2];
    a.T1 = out[3];
    a.acc = acc;
    a.objective = c->objective;
    a.beta = rp<R>(c->beta);
    return a;
  }

  // two time steps per launch: FP32 D2Q9 sweeps (the adjoint ones steady),
  // and the FP64 non-thermal forward sweep (two-step kernels exist for 64 x 4
  // and 64 x 8 tiles)
  bool two_step(int spl) const {
    return std::is_same<R, float>::value && c->dim == 2 && spl == 2 &&
           (c->geo.ty == 4 || c->geo.ty == 8);
  }
  bool two_step_fwd(int spl) const {
    return two_step(spl) || (c->dim == 2 && spl == 2 && !c->phys.thermal &&
                             (c->geo.ty == 4 || c->geo.ty == 8));
  }

  void coefficients(const double* gamma) {
    const double Kf = c->phys.thermal ? c->phys.nu / c->phys.Pr : 0.0;
    const double Ks = Kf * (c->phys.thermal ? c->phys.Ks_over_Kf : 1.0);
    const double qK = c->phys.thermal ? c->phys.q_K : 1.0;
    if (c->dim == 3)
      lks::launch_coef3<R>(c->geo3, c->d_mask, gamma, c->phys.alpha_max, c->phys.q_alpha, Kf, Ks,
                           qK, rp<R>(c->inv1pa), rp<R>(c->B), rp<R>(c->dA3), rp<R>(c->dB),
                           c->stream);
    else
      lks::launch_coef<R>(g, gamma, c->phys.alpha_max, c->phys.q_alpha, Kf, Ks, qK,
                          rp<R>(c->inv1pa), rp<R>(c->B), rp<R>(c->dA3), rp<R>(c->dB), c->stream);
    if (has_source(c))
      lks::launch_source_coef<R>(g, gamma, c->phys.beta_max, c->phys.q_beta, rp<R>(c->beta),
                                 rp<R>(c->dbeta), c->stream);
  }

  void init(R* const s[5]) {
    if (c->dim == 3) {
      const R* ub[3] = {rp<R>(c->ubx), rp<R>(c->uby), rp<R>(c->ubz)};
      lks::launch_init3<R>(c->geo3, c->d_mask, ub, rp<R>(c->Tb), c->ufac[0], s, c->stream);
      return;
    }
    lks::launch_init<R>(g, c->d_mask, rp<R>(c->ubx), rp<R>(c->uby), rp<R>(c->Tb), c->ufac[0],
                        s[0], s[1], s[2], s[3], c->stream);
  }

  // binomial checkpointing: snapshot j (the layout of a checkpoint) and the
  // ping-pong working buffers p
  void snap(int j, R* out[5]) {
    for (int f = 0; f < 5; ++f) out[f] = f < ckpt_fields(c) ? ckpt(j, f) : nullptr;
  }
  void work(int p, R* out[5]) {
    for (int f = 0; f < 5; ++f) out[f] = f < nf ? rp<R>(c->S[p][f]) : nullptr;
    if (!c->phys.thermal) out[nf - 1] = nullptr;
  }
  // `steps` LKS steps from level `from` held in `in`; the last step writes
  // `last` when given, the others alternate between the working buffers.
  // res receives the pointers of the final level.
  void bin_advance(R* const in[5], int from, int steps, R* const* last, R* res[5], double* acc) {
    R* cur[5];
    for (int f = 0; f < 5; ++f) cur[f] = in[f];
    int p = 0;
    for (int i = 0; i < steps; ++i) {
      R* out[5];
      if (last && i == steps - 1) {
        for (int f = 0; f < 5; ++f) out[f] = last[f];
      } else {
        work(p, out);
        p ^= 1;
      }
      step(cur, out, from + i + 1, acc);
      for (int f = 0; f < 5; ++f) cur[f] = out[f];
    }
    for (int f = 0; f < 5; ++f) res[f] = cur[f];
  }

  // forward sweep of a binomial plan: level 0 in snapshot 0, the leading
  // placements of the schedule on the way, the objective over every level
  void forward_binomial(int steps) {
    R* cur[5];
    snap(0, cur);
    init(cur);
    int lvl = 0;
    const Plan& p = c->plan;
    for (int i = 0; i < p.n_pre; ++i) {
      const Act& x = p.acts[size_t(i)];
      R* dst[5];
      snap(x.dst, dst);
      bin_advance(cur, lvl, x.steps, dst, cur, c->acc);
      lvl += x.steps;
    }
    bin_advance(cur, lvl, steps - lvl, nullptr, cur, c->acc);
    for (int f = 0; f < 5; ++f) c->lastv[f] = cur[f];
    lks::launch_finite_check<R>(cur[1], N, c->flag, c->stream);
    c->last_level = steps;
  }

  void forward(const double* gamma, int steps) {
    coefficients(gamma);
    if (c->mode == LKS_UNSTEADY && c->plan.scheme == LKS_CKPT_BINOMIAL) {
      lks::launch_fill(c->acc, size_t(acc_count(c)), 0.0, c->stream);
      forward_binomial(steps);
      return;
    }
    if (c->mode == LKS_STEADY) {
      R* s0[5] = {};
      for (int f = 0; f < nf; ++f) s0[f] = rp<R>(c->S[0][f]);
      init(s0);
      c->cur = 0;
      advance(steps);
      return;
    }
    lks::launch_fill(c->acc, size_t(acc_count(c)), 0.0, c->stream);
    R* lv[5];
    level(0, c->plan.ls, lv);
    init(lv);
    R* last[5];
    sweep(0, steps, c->plan.ls, c->acc, last);
    for (int f = 0; f < 5; ++f) c->lastv[f] = last[f];
    lks::launch_finite_check<R>(last[1], N, c->flag, c->stream);
    c->last_level = steps;
  }

  void advance(int steps) {
    int n = 0;
    if (two_step_fwd(c->spl_f)) {
      for (; n + 2 <= steps; n += 2) {
        R* in[5] = {};
        R* out[5] = {};
        for (int f = 0; f < nf; ++f) {
          in[f] = rp<R>(c->S[c->cur][f]);
          out[f] = rp<R>(c->S[c->cur ^ 1][f]);
        }
        lks::launch_lks_step2(g, fwd_args(in, out, c->last_level + n + 2, nullptr), c->stream);
        c->cur ^= 1;
      }
    }
    for (; n < steps; ++n) {
      R* in[5] = {};
      R* out[5] = {};
      for (int f = 0; f < nf; ++f) {
        in[f] = rp<R>(c->S[c->cur][f]);
        out[f] = rp<R>(c->S[c->cur ^ 1][f]);
      }
      step(in, out, c->last_level + n + 1, nullptr);
      c->cur ^= 1;
    }
    c->last_level += steps;
    lks::launch_finite_check<R>(cur_field(1), N, c->flag, c->stream);
    if (c->objective == LKS_OBJ_PRESSURE_DROP) {
      if (c->dim == 3)
        lks::launch_tag_sum3<R>(c->geo3, c->d_mask, cur_field(0), cur_field(1), cur_field(4),
                                LKS_OBJ_PRESSURE_DROP, c->acc, c->scal, c->stream);
      else
        lks::launch_pressure_drop<R>(g, c->d_mask, cur_field(0), c->scal, c->stream);
    } else if (c->objective == LKS_OBJ_HEAT_EXCHANGE) {
      lks::launch_source_heat<R>(g, rp<R>(c->beta), cur_field(3), c->scal, c->stream);
    } else if (c->objective == LKS_OBJ_HEAT_SINK) {
      lks::launch_probe_T<R>(g, c->d_mask, cur_field(3), c->scal, c->stream);
    } else {
      probe_heat_steady();
    }
  }

  void probe_heat_steady() {
    if (c->dim == 3)
      lks::launch_tag_sum3<R>(c->geo3, c->d_mask, cur_field(0), cur_field(1), cur_field(4),
                              LKS_OBJ_HEAT, c->acc, c->scal, c->stream);
    else
      lks::launch_probe_heat<R>(g, c->d_mask, cur_field(1), cur_field(3), c->scal, c->stream);
  }

  void zero_adjoint(int which) {
    for (int f = 0; f < nf; ++f) lks::launch_fill_r<R>(rp<R>(c->P[which][f]), N, c->stream);
  }

  // one ALKS step with the state st (drho, u..., T) of the destination level
  // seeds of one level for objective weight w: pressure drop, probe heat,
  // heat exchange, heated boundary (per node)
  void seeds(double w, double* sdp, double* sh, double* ss, double* sbt) const {
    *sdp = c->objective == LKS_OBJ_PRESSURE_DROP ? w : 0.0;
    *sh = c->objective == LKS_OBJ_HEAT ? w : 0.0;
    *ss = c->objective == LKS_OBJ_HEAT_EXCHANGE ? w : 0.0;
    *sbt = c->objective == LKS_OBJ_HEAT_SINK ? w / std::max(c->n_probe, 1) : 0.0;
  }

  // b_only: exact mode at level 0, where the sensitivity keeps the
  // conductivity term only
  void adj_step(R* const st[5], double sdp, double sh, double* sens, int mode, double ss = 0.0,
                double sbt = 0.0, bool b_only = false) {
    const int i0 = c->acur, i1 = c->acur ^ 1;
    if (c->dim == 3) {
      lks::Adj3Args<R> a;
      a.mask = c->d_mask;
      a.inv1pa = rp<R>(c->inv1pa);
      a.B = rp<R>(c->B);
      a.dA3 = rp<R>(c->dA3);
      a.dB = rp<R>(c->dB);
      a.u[0] = st[1];
      a.u[1] = st[2];
      a.u[2] = st[3];
      a.T = st[4] ? st[4] : st[1];
      for (int f = 0; f < 5; ++f) {
        a.p0[f] = rp<R>(c->P[i0][f]);
        a.p1[f] = rp<R>(c->P[i1][f]);
      }
      a.m = rp<R>(c->M3);
      a.ops = static_cast<const lks::FaceOpT<R>*>(c->d_ops3);
      a.face = c->face3;
      a.nface = int(c->face3h.size());
      a.sens = sens;
      a.sens_mode = sens ? mode : 0;
      a.exact = c->adj_exact;
      a.seed_dp = sdp;
      a.seed_heat = sh;
      a.sens_b_only = b_only ? 1 : 0;
      lks::launch_alks3_step<R>(c->geo3, a, c->stream);
      c->acur = i1;
      return;
    }
    lks::AdjArgs<R> a = adj_args(st, sdp, sh, sens, mode);
    a.seed_src = ss;
    a.seed_bt = sbt;
    a.sens_b_only = b_only ? 1 : 0;
    lks::launch_alks_step<R>(g, a, c->stream);
    c->acur = i1;
  }

  lks::AdjArgs<R> adj_args(R* const st[5], double sdp, double sh, double* sens, int mode) {
    const int i0 = c->acur, i1 = c->acur ^ 1;
    lks::AdjArgs<R> a;
    a.mask = c->d_mask;
    a.inv1pa = rp<R>(c->inv1pa);
    a.B = rp<R>(c->B);
    a.dA3 = rp<R>(c->dA3);
    a.dB = rp<R>(c->dB);
    a.ux = st[1];
    a.uy = st[2];
    a.T = st[3] ? st[3] : st[1];
    a.r0 = rp<R>(c->P[i0][0]);
    a.vx0 = rp<R>(c->P[i0][1]);
    a.vy0 = rp<R>(c->P[i0][2]);
    a.th0 = rp<R>(c->P[i0][3]);
    a.r1 = rp<R>(c->P[i1][0]);
    a.vx1 = rp<R>(c->P[i1][1]);
    a.vy1 = rp<R>(c->P[i1][2]);
    a.th1 = rp<R>(c->P[i1][3]);
    a.sens = sens;
    a.sens_mode = sens ? mode : 0;
    a.exact = c->adj_exact;
    a.seed_dp = sdp;
    a.seed_heat = sh;
    a.ops = static_cast<const lks::RingOpT<R>*>(c->d_ops);
    a.beta = rp<R>(c->beta);
    a.dbeta = rp<R>(c->dbeta);
    return a;
  }

  void adjoint_steady(double seed, int steps, double* dJ, bool reset) {
    if (reset) {
      c->acur = 0;
      zero_adjoint(0);
    }
    double sdp, sh, ss, sbt;
    seeds(seed, &sdp, &sh, &ss, &sbt);
    R* st[5] = {};
    for (int f = 0; f < nf; ++f) st[f] = cur_field(f);
    if (!c->phys.thermal) st[nf - 1] = nullptr;
    int n = 0;
    if constexpr (std::is_same<R, float>::value) {
      if (two_step(c->spl_a) && steps >= 2) {
        if (steps % 2) adj_step(st, sdp, sh, nullptr, 2, ss, sbt);
        for (n = steps % 2; n < steps; n += 2) {
          lks::AdjArgs<R> a = adj_args(st, sdp, sh, n + 2 == steps ? dJ : nullptr, 2);
          a.seed_src = ss;
          a.seed_bt = sbt;
          lks::launch_alks_step2(g, a, c->stream);
          c->acur ^= 1;
        }
      }
    }
    for (; n < steps; ++n) {
      const bool last = n == steps - 1;
      adj_step(st, sdp, sh, last ? dJ : nullptr, 2, ss, sbt);
    }
  }

  // reverse sweep of a binomial plan: the schedule's actions after the
  // placements the forward sweep made
  void adjoint_binomial(double seed, double* dJ) {
    const int Nst = c->n_steps;
    const Plan& p = c->plan;
    lks::launch_fill(dJ, N, 0.0, c->stream);
    c->acur = 0;
    zero_adjoint(0);
    R* wk[5] = {};
    for (size_t i = size_t(p.n_pre); i < p.acts.size(); ++i) {
      const Act& x = p.acts[i];
      R* src[5];
      snap(x.src >= 0 ? x.src : 0, src);
      if (!x.adjoint) {
        R* dst[5];
        if (x.dst >= 0) snap(x.dst, dst);
        bin_advance(src, x.from, x.steps, x.dst >= 0 ? dst : nullptr, wk, nullptr);
        continue;
      }
      R* const* lv = x.src >= 0 ? src : wk;
      const int n = x.from;
      double sdp, sh, ss, sbt;
      seeds(n >= 1 ? seed / Nst : 0.0, &sdp, &sh, &ss, &sbt);
      adj_step(lv, sdp, sh, dJ, 1, ss, sbt, n == 0 && c->adj_exact);
    }
  }

  void adjoint_unsteady(double seed, double* dJ) {
    if (c->plan.scheme == LKS_CKPT_BINOMIAL) {
      adjoint_binomial(seed, dJ);
      return;
    }
    const int Nst = c->n_steps, K = c->plan.K;
    lks::launch_fill(dJ, N, 0.0, c->stream);
    c->acur = 0;
    zero_adjoint(0);
    for (int b = c->plan.ls; b >= 0; b -= K) {
      const int top = (b == c->plan.ls) ? Nst : b + K - 1;
      if (b != c->plan.ls) {
        // replay levels b+1 .. top into the segment slots
        R* last[5];
        sweep(b, top, b, nullptr, last);
      }
      for (int n = top; n >= b; --n) {
        R* lv[5];
        level(n, b, lv);
        double sdp, sh, ss, sbt;
        seeds(n >= 1 ? seed / Nst : 0.0, &sdp, &sh, &ss, &sbt);
        // the exact mode pairs the Brinkman and source terms with the levels
        // the steps produce (1..N; the initial state does not depend on
        // gamma) and the conductivity term with the equilibria the steps use
        adj_step(lv, sdp, sh, dJ, 1, ss, sbt, n == 0 && c->adj_exact);
      }
    }
  }

  // internal index of a forward field id, or -1
  int fwd_index(int which) {
    if (which == LKS_FIELD_DRHO || which == LKS_FIELD_UX || which == LKS_FIELD_UY) return which;
    if (which == LKS_FIELD_T) return c->phys.thermal ? nf - 1 : -1;
    if (which == LKS_FIELD_UZ) return c->dim == 3 ? 3 : -1;
    return -1;
  }
  int adj_index(int which) {
    if (which == LKS_FIELD_ADJ_RHO || which == LKS_FIELD_ADJ_VX || which == LKS_FIELD_ADJ_VY)
      return which - LKS_FIELD_ADJ_RHO;
    if (which == LKS_FIELD_ADJ_THETA) return c->phys.thermal ? nf - 1 : -1;
    if (which == LKS_FIELD_ADJ_VZ) return c->dim == 3 ? 3 : -1;
    return -1;
  }

  lks_status read(int which, double* out) {
    const void* src = nullptr;
    int f;
    if ((f = fwd_index(which)) >= 0) {
      if (c->mode == LKS_STEADY) {
        src = c->S[c->cur][f];
      } else {
        // the final level of the forward sweep (the sweeps track where its
        // ping-pong fields are)
        src = c->lastv[f];
      }
    } else if ((f = adj_index(which)) >= 0) {
      src = c->P[c->acur][f];
    } else {
      return LKS_E_INVALID;
    }
    if (!src) return LKS_E_STATE;  // no unsteady forward sweep on this workspace yet
    lks::launch_to_double<R>(static_cast<const R*>(src), out, N, c->stream);
    return LKS_OK;
  }

  lks_status write(int which, const double* in) {
    void* dst = nullptr;
    int f;
    if ((f = fwd_index(which)) >= 0) {
      if (c->mode != LKS_STEADY) return LKS_E_UNSUPPORTED;
      dst = c->S[c->cur][f];
    } else if ((f = adj_index(which)) >= 0) {
      dst = c->P[c->acur][f];
    } else {
      return LKS_E_INVALID;
    }
    lks::launch_from_double<R>(in, static_cast<R*>(dst), N, c->stream);
    return LKS_OK;
  }
};

lks_status check_launch(lks_ctx* c) {
  hipError_t e = hipGetLastError();
  lks_status st = LKS_OK;
  hip_ok(c, e, "kernel launch", &st);
  return st;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

lks_status lks_create(const lks_grid* grid, const lks_phys* phys, const lks_bc* bc,
                      size_t mem_budget_bytes, void* hip_stream, lks_ctx** out) {
  if (!out) return fail(nullptr, LKS_E_INVALID, "null output pointer");
  *out = nullptr;
  if (!grid || !phys || !bc) return fail(nullptr, LKS_E_INVALID, "null descriptor");
  if (grid->precision == LKS_MIXED) {
    // an FP64 context for the forward sweep with an FP32 context for the
    // adjoint sweep of the same problem
    if (grid->lattice != LKS_D2Q9 || bc->mode != LKS_STEADY)
      return fail(nullptr, LKS_E_UNSUPPORTED, "mixed precision applies to steady D2Q9 problems");
    lks_grid g64 = *grid, g32 = *grid;
    g64.precision = LKS_FP64;
    g32.precision = LKS_FP32DEV;
    lks_ctx* hi = nullptr;
    lks_ctx* lo = nullptr;
    lks_status st = lks_create(&g64, phys, bc, mem_budget_bytes, hip_stream, &hi);
    if (st != LKS_OK) return st;
    st = lks_create(&g32, phys, bc, mem_budget_bytes, hip_stream, &lo);
    if (st != LKS_OK) {
      lks_destroy(hi);
      return st;
    }
    hi->lo = lo;
    *out = hi;
    return LKS_OK;
  }
  const bool d3 = grid->lattice == LKS_D3Q19;
  lks_status st = d3 ? validate3(grid, phys, bc) : validate(grid, phys, bc);
  if (st != LKS_OK) return st;
  lks_ctx* c = new lks_ctx();
  c->grid = *grid;
  if (!d3) c->grid.nz = 1;
  c->dim = d3 ? 3 : 2;
  c->phys = *phys;
  c->objective = bc->objective;
  c->mode = bc->mode;
  c->n_steps = bc->mode == LKS_UNSTEADY ? bc->n_steps : 0;
  c->rho_out = bc->rho_out;
  const int N = grid->nx * grid->ny * c->grid.nz;
  c->N = N;
  c->mask.assign(bc->node_class, bc->node_class + N);
  if (d3 ? grid->periodic == 7 : grid->periodic != 0)
    for (auto& m : c->mask) m &= uint8_t(~15);
  c->ubar.assign(bc->u_bar, bc->u_bar + size_t(c->dim) * N);
  if (bc->T_bar) c->Tbar.assign(bc->T_bar, bc->T_bar + N);
  else c->Tbar.assign(N, 0.0);
  if (bc->u_factor) c->ufac.assign(bc->u_factor, bc->u_factor + bc->n_factor);
  else c->ufac.assign(1, 1.0);
  for (int k = 0; k < N; ++k) {
    if (c->mask[k] & LKS_TAG_PROBE) ++c->n_probe;
    if (c->mask[k] & LKS_TAG_J_INLET) ++c->n_in;
    if (c->mask[k] & LKS_TAG_J_OUTLET) ++c->n_out;
  }
  Geo& g = c->geo;
  g.nx = grid->nx;
  g.ny = grid->ny;
  g.N = N;
  g.periodic = grid->periodic ? 1 : 0;
  g.thermal = phys->thermal ? 1 : 0;
  // thermal tiles hold twice the LDS arrays; 64 x 4 tiles keep more blocks
  // resident per CU (the autotuner may still choose another height)
  set_tile_rows(g, phys->thermal ? 4 : 8);
  g.A = 4.5 * (1.0 / 6.0 - phys->nu);
  const double Kf = phys->thermal ? phys->nu / phys->Pr : 0.0;
  g.Bf = 3.0 * (1.0 / 6.0 - Kf);
  g.drho_out = bc->rho_out - 1.0;
  g.gbx = phys->gbeta[0];
  g.gby = phys->gbeta[1];
  g.Tref = phys->T_ref;
  lks::build_ring_ops(g.A, g.Bf, c->ops);
  if (d3) {
    lks::Geo3& g3 = c->geo3;
    g3.nx = grid->nx;
    g3.ny = grid->ny;
    g3.nz = grid->nz;
    g3.N = N;
    g3.periodic = grid->periodic;
    g3.thermal = g.thermal;
    g3.A = g.A;
    g3.Bf = g.Bf;
    g3.drho_out = g.drho_out;
    g3.zc = g3.zca = g3.zcf = 16;  // re-planned for the device at bind
    g3.fused = 1;
    lks::build_face_ops3(g3.A, g3.Bf, c->ops3);
    c->copy3h.resize(size_t(lks::copy_nodes3(g3, nullptr)));
    lks::copy_nodes3(g3, c->copy3h.data());
    c->face3h.resize(size_t(lks::face_nodes3(g3, nullptr)));
    lks::face_nodes3(g3, c->face3h.data());
  }
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->budget = mem_budget_bytes;
  c->rsz = grid->precision == LKS_FP64 ? 8 : 4;
  st = plan_memory(c);
  if (st != LKS_OK) {
    delete c;
    return st;
  }
  *out = c;
  return LKS_OK;
}

}  // extern "C"

// The allocation-free workspace: one array per device, loaded with the code
// object and held until the process ends. Host code never passes the array's
// name to a kernel (on the host it is a stand-in, not a device address); it
// asks for the device address once per device and uses that.
namespace {
static __device__ __align__(256) unsigned char scratch[LKS_STATIC_WORKSPACE_BYTES];

struct StaticScratch {
  void* ptr = nullptr;            // device address of `scratch` on the device
  const lks_ctx* owner = nullptr;  // context bound to it last
};
std::mutex g_scratch_mu;
std::map<int, StaticScratch> g_scratch;  // by device ordinal
}  // namespace

// workspace of a context, including the FP32 adjoint context of a mixed one
static size_t ws_total(const lks_ctx* c) {
  return c->lo ? align256(c->plan.total) + c->lo->plan.total : c->plan.total;
}

extern "C" {

lks_status lks_workspace_size(const lks_ctx* c, size_t* bytes) {
  if (!c || !bytes) return LKS_E_INVALID;
  *bytes = ws_total(c);
  return LKS_OK;
}

lks_status lks_bind_workspace(lks_ctx* c, void* dev_ptr, size_t bytes) {
  if (!c) return LKS_E_INVALID;
  if (!dev_ptr) return fail(c, LKS_E_INVALID, "null workspace");
  if (reinterpret_cast<uintptr_t>(dev_ptr) & 255)
    return fail(c, LKS_E_INVALID, "workspace must be 256-byte aligned");
  if (bytes < ws_total(c)) return fail(c, LKS_E_NOMEM, "workspace smaller than lks_workspace_size");
  if (c->lo) {
    // mixed precision: the FP32 adjoint context takes the tail
    const size_t hi = align256(c->plan.total);
    lks_status st = lks_bind_workspace(c->lo, static_cast<char*>(dev_ptr) + hi, bytes - hi);
    if (st != LKS_OK) return fail(c, st, std::string("adjoint part: ") + c->lo->err);
    bytes = c->plan.total;
  }
  const size_t N = size_t(c->N), r = size_t(c->rsz);
  const int nf = nfields(c), nu = c->dim;
  char* p = static_cast<char*>(dev_ptr);
  auto take = [&](size_t b) {
    char* q = p;
    p += align256(b);
    return q;
  };
  c->ws = static_cast<char*>(dev_ptr);
  c->ws_bytes = bytes;
  if (c->dim == 3) lks::zplan3(c->geo3, int(c->rsz));
  c->d_mask = reinterpret_cast<uint8_t*>(take(N));
  c->ubx = take(N * r);
  c->uby = take(N * r);
  c->ubz = nu == 3 ? take(N * r) : nullptr;
  c->Tb = take(N * r);
  c->d_ufac = reinterpret_cast<double*>(take(sizeof(double) * c->ufac.size()));
  c->inv1pa = take(N * r);
  c->B = take(N * r);
  c->dA3 = take(N * r);
  c->dB = take(N * r);
  if (has_source(c)) {
    c->beta = take(N * r);
    c->dbeta = take(N * r);
  }
  for (int s = 0; s < 2; ++s)
    for (int f = 0; f < 5; ++f) c->S[s][f] = f < nf ? take(N * r) : nullptr;
  for (int s = 0; s < 2; ++s)
    for (int f = 0; f < 5; ++f) c->P[s][f] = f < nf ? take(N * r) : nullptr;
  for (auto& p : c->lastv) p = nullptr;
  c->acc = reinterpret_cast<double*>(take(sizeof(double) * acc_capacity(c)));
  if (nu == 3) {
    c->d_ops3 = take(6 * sizeof(lks::FaceOp3));
    c->copy3 = reinterpret_cast<int*>(take(sizeof(int) * c->copy3h.size()));
    c->face3 = reinterpret_cast<int*>(take(sizeof(int) * c->face3h.size()));
    c->M3 = take(size_t(moments3_fields(c)) * N * r);
  } else {
    c->d_ops = take(4 * sizeof(lks::RingOp));
  }
  c->scal = reinterpret_cast<double*>(take(sizeof(double) * 8));
  c->flag = reinterpret_cast<int*>(take(sizeof(int) * 4));
  if (c->mode == LKS_UNSTEADY) {
    c->C = take(size_t(c->plan.n_ckpt) * ckpt_fields(c) * N * r);
    c->Seg = take(size_t(c->plan.n_slots) * slot_fields(c) * N * r);
  }
  // upload boundary data in the working precision: u_bar blocks, then T_bar
  lks_status st = LKS_OK;
  std::vector<char> tmp(size_t(nu + 1) * N * r);
  for (int b = 0; b <= nu; ++b) {
    const double* src = b < nu ? c->ubar.data() + size_t(b) * N : c->Tbar.data();
    for (size_t k = 0; k < N; ++k) {
      if (r == 8) reinterpret_cast<double*>(tmp.data())[size_t(b) * N + k] = src[k];
      else reinterpret_cast<float*>(tmp.data())[size_t(b) * N + k] = float(src[k]);
    }
  }
  void* dst[4] = {c->ubx, c->uby, nu == 3 ? c->ubz : c->Tb, c->Tb};
  if (!hip_ok(c, hipMemcpyAsync(c->d_mask, c->mask.data(), N, hipMemcpyHostToDevice, c->stream),
              "upload mask", &st))
    return st;
  for (int b = 0; b <= nu; ++b)
    if (!hip_ok(c, hipMemcpyAsync(dst[b], tmp.data() + size_t(b) * N * r, N * r,
                                  hipMemcpyHostToDevice, c->stream),
                "upload boundary values", &st))
      return st;
  // the operators in the arithmetic type of the kernels
  const bool f32 = c->rsz == 4;
  if (f32) {
    for (int o = 0; o < 4; ++o) c->ops_f[o] = lks::ring_op_as<float>(c->ops[o]);
    for (int o = 0; o < 6; ++o) c->ops3_f[o] = lks::face_op_as<float>(c->ops3[o]);
  }
  const void* ops_src = f32 ? static_cast<const void*>(c->ops_f) : static_cast<const void*>(c->ops);
  const size_t ops_bytes = f32 ? sizeof c->ops_f : sizeof c->ops;
  const void* ops3_src =
      f32 ? static_cast<const void*>(c->ops3_f) : static_cast<const void*>(c->ops3);
  const size_t ops3_bytes = f32 ? sizeof c->ops3_f : sizeof c->ops3;
  const bool ops_ok = nu == 3
      ? hip_ok(c, hipMemcpyAsync(c->d_ops3, ops3_src, ops3_bytes, hipMemcpyHostToDevice,
                                 c->stream), "upload face operators", &st) &&
            hip_ok(c, hipMemcpyAsync(c->copy3, c->copy3h.data(), sizeof(int) * c->copy3h.size(),
                                     hipMemcpyHostToDevice, c->stream),
                   "upload edge nodes", &st) &&
            hip_ok(c, hipMemcpyAsync(c->face3, c->face3h.data(), sizeof(int) * c->face3h.size(),
                                     hipMemcpyHostToDevice, c->stream),
                   "upload boundary nodes", &st)
      : hip_ok(c, hipMemcpyAsync(c->d_ops, ops_src, ops_bytes, hipMemcpyHostToDevice, c->stream),
               "upload ring operators", &st);
  if (!ops_ok ||
      !hip_ok(c, hipMemcpyAsync(c->d_ufac, c->ufac.data(), sizeof(double) * c->ufac.size(),
                                hipMemcpyHostToDevice, c->stream),
              "upload u_factor", &st) ||
      !hip_ok(c, hipStreamSynchronize(c->stream), "bind sync", &st))
    return st;
  // clear the state so that an unused thermal field reads as zero
  for (int s = 0; s < 2; ++s)
    for (int f = 0; f < nf; ++f) {
      if (r == 8) lks::launch_fill_r<double>(static_cast<double*>(c->S[s][f]), N, c->stream);
      else lks::launch_fill_r<float>(static_cast<float*>(c->S[s][f]), N, c->stream);
    }
  int zero[4] = {0, 0, 0, 0};
  if (!hip_ok(c, hipMemcpyAsync(c->flag, zero, sizeof zero, hipMemcpyHostToDevice, c->stream),
              "clear flag", &st) ||
      !hip_ok(c, hipStreamSynchronize(c->stream), "bind sync", &st))
    return st;
  c->bound = true;
  c->static_dev = -1;
  c->have_forward = false;
  c->have_adjoint = false;
  return check_launch(c);
}

lks_status lks_bind_static_workspace(lks_ctx* c) {
  if (!c) return LKS_E_INVALID;
  if (ws_total(c) > size_t(LKS_STATIC_WORKSPACE_BYTES)) {
    char buf[160];
    snprintf(buf, sizeof buf, "workspace of %zu B exceeds the static array of %zu B",
             ws_total(c), size_t(LKS_STATIC_WORKSPACE_BYTES));
    return fail(c, LKS_E_NOMEM, buf);
  }
  lks_status st = LKS_OK;
  int dev = 0;
  if (!hip_ok(c, hipGetDevice(&dev), "current device", &st)) return st;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  StaticScratch& sc = g_scratch[dev];
  if (!sc.ptr) {
    void* ptr = nullptr;
    if (!hip_ok(c, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "static workspace address",
                &st))
      return st;
    if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & 255))
      return fail(c, LKS_E_HIP, "static workspace address is null or misaligned");
    sc.ptr = ptr;
  }
  // the previous context of this device loses the array: its state is gone
  if (sc.owner && sc.owner != c) {
    lks_ctx* prev = const_cast<lks_ctx*>(sc.owner);
    prev->bound = false;
    prev->have_forward = false;
    prev->have_adjoint = false;
  }
  sc.owner = nullptr;
  st = lks_bind_workspace(c, sc.ptr, size_t(LKS_STATIC_WORKSPACE_BYTES));
  if (st != LKS_OK) return st;
  c->static_dev = dev;
  sc.owner = c;
  return LKS_OK;
}

static lks_status forward_impl(lks_ctx* c, const double* gamma, int steps, bool reset) {
  if (!c) return LKS_E_INVALID;
  if (!c->bound) return fail(c, LKS_E_STATE, unbound_reason(c));
  if (!gamma) return fail(c, LKS_E_INVALID, "null gamma");
  if (steps < 0) return fail(c, LKS_E_INVALID, "negative step count");
  if (c->mode == LKS_UNSTEADY) {
    if (!reset) return fail(c, LKS_E_UNSUPPORTED, "advance applies to steady problems");
    if (steps != c->n_steps) return fail(c, LKS_E_INVALID, "unsteady forward needs steps == n_steps");
  } else if (!reset && !c->have_forward) {
    return fail(c, LKS_E_STATE, "advance before forward");
  }
  if (reset) {
    c->last_level = 0;
    lks::launch_clear_flag(c->flag, c->stream);  // the divergence flag of this run
  }
  if (c->rsz == 8) {
    Run<double> r(c);
    if (reset) r.forward(gamma, steps);
    else { r.coefficients(gamma); r.advance(steps); }
  } else {
    Run<float> r(c);
    if (reset) r.forward(gamma, steps);
    else { r.coefficients(gamma); r.advance(steps); }
  }
  lks_status st = check_launch(c);
  if (st == LKS_OK) {
    c->have_forward = true;
    c->have_adjoint = false;
    if (c->lo) {
      // mixed: the FP32 adjoint part takes the design coefficients now
      if (!c->lo->bound) return fail(c, LKS_E_STATE, "adjoint part not bound");
      Run<float>(c->lo).coefficients(gamma);
      c->lo->have_adjoint = false;
      st = check_launch(c);
    }
  }
  return st;
}

lks_status lks_forward(lks_ctx* c, const double* gamma_dev, int steps) {
  return forward_impl(c, gamma_dev, steps, true);
}

lks_status lks_advance(lks_ctx* c, const double* gamma_dev, int steps) {
  return forward_impl(c, gamma_dev, steps, false);
}

lks_status lks_objective(lks_ctx* c, double* J) {
  if (!c || !J) return LKS_E_INVALID;
  if (!c->have_forward) return fail(c, LKS_E_STATE, "objective before forward");
  lks_status st = LKS_OK;
  double sc[8];
  int flag[4];
  if (c->mode == LKS_UNSTEADY) lks::launch_sum(c->acc, acc_count(c), c->scal, c->stream);
  if (!hip_ok(c, hipMemcpyAsync(sc, c->scal, sizeof sc, hipMemcpyDeviceToHost, c->stream),
              "read objective", &st) ||
      !hip_ok(c, hipMemcpyAsync(flag, c->flag, sizeof flag, hipMemcpyDeviceToHost, c->stream),
              "read flag", &st) ||
      !hip_ok(c, hipStreamSynchronize(c->stream), "objective sync", &st))
    return st;
  if (flag[0]) return fail(c, LKS_E_DIVERGED, "non-finite velocity in the forward state");
  const double s = sc[0];
  if (c->objective == LKS_OBJ_PRESSURE_DROP) {
    if (c->mode == LKS_UNSTEADY)
      *J = (s / c->n_steps + double(c->n_in - c->n_out)) / 3.0;
    else
      *J = (s + double(c->n_in - c->n_out)) / 3.0;
  } else {
    const double per = c->objective == LKS_OBJ_HEAT_SINK ? double(std::max(c->n_probe, 1)) : 1.0;
    *J = (c->mode == LKS_UNSTEADY ? s / c->n_steps : s) / per;
  }
  return LKS_OK;
}

static lks_status backward_impl(lks_ctx* c, double seed, int steps, double* dJ, bool reset) {
  if (!c) return LKS_E_INVALID;
  if (!c->have_forward) return fail(c, LKS_E_STATE, "alks_backward before lks_forward");
  if (c->lo) {
    // mixed precision: the FP32 context takes the design coefficients and the
    // final FP64 forward state rounded to float, then runs the adjoint
    lks_ctx* lo = c->lo;
    if (reset) {
      if (!lo->bound) return fail(c, LKS_E_STATE, "adjoint part not bound");
      const int nf = nfields(c);
      for (int f = 0; f < nf; ++f)
        lks::launch_from_double<float>(static_cast<const double*>(c->S[c->cur][f]),
                                       static_cast<float*>(lo->S[lo->cur][f]), c->N, c->stream);
      lo->have_forward = true;
      lo->have_adjoint = false;
    }
    lks_status st = backward_impl(lo, seed, steps, dJ, reset);
    if (st != LKS_OK) return fail(c, st, lo->err);
    c->have_adjoint = true;
    return LKS_OK;
  }
  if (!std::isfinite(seed)) return fail(c, LKS_E_INVALID, "seed not finite");
  if (c->mode == LKS_UNSTEADY) {
    if (!reset) return fail(c, LKS_E_UNSUPPORTED, "alks_advance applies to steady problems");
    if (!dJ) return fail(c, LKS_E_INVALID, "null dJ/dgamma");
  } else {
    if (steps < 1) return fail(c, LKS_E_INVALID, "steady adjoint needs adj_steps >= 1");
    if (reset && !dJ) return fail(c, LKS_E_INVALID, "null dJ/dgamma");
    if (!reset && !c->have_adjoint) return fail(c, LKS_E_STATE, "alks_advance before alks_backward");
  }
  if (c->rsz == 8) {
    Run<double> r(c);
    if (c->mode == LKS_UNSTEADY) r.adjoint_unsteady(seed, dJ);
    else r.adjoint_steady(seed, steps, dJ, reset);
  } else {
    Run<float> r(c);
    if (c->mode == LKS_UNSTEADY) r.adjoint_unsteady(seed, dJ);
    else r.adjoint_steady(seed, steps, dJ, reset);
  }
  // flag[1]: a non-finite sensitivity in the last adjoint sweep
  lks::launch_clear_flag(c->flag + 1, c->stream);
  if (dJ) lks::launch_finite_check<double>(dJ, size_t(c->N), c->flag + 1, c->stream);
  lks_status st = check_launch(c);
  if (st == LKS_OK) c->have_adjoint = true;
  return st;
}

lks_status lks_gradient_status(lks_ctx* c) {
  if (!c) return LKS_E_INVALID;
  if (!c->have_adjoint) return fail(c, LKS_E_STATE, "gradient status before alks_backward");
  lks_status st = LKS_OK;
  int flag[4];
  if (!hip_ok(c, hipMemcpyAsync(flag, c->flag, sizeof flag, hipMemcpyDeviceToHost, c->stream),
              "read flag", &st) ||
      !hip_ok(c, hipStreamSynchronize(c->stream), "gradient status sync", &st))
    return st;
  if (flag[0]) return fail(c, LKS_E_DIVERGED, "non-finite velocity in the forward state");
  if (c->lo) {
    st = lks_gradient_status(c->lo);
    return st == LKS_OK ? st : fail(c, st, c->lo->err);
  }
  if (flag[1]) return fail(c, LKS_E_DIVERGED, "non-finite sensitivity in the adjoint sweep");
  return LKS_OK;
}

lks_status alks_backward(lks_ctx* c, double J_seed, int adj_steps, double* dJdgamma_dev) {
  return backward_impl(c, J_seed, adj_steps, dJdgamma_dev, true);
}

lks_status alks_advance(lks_ctx* c, double J_seed, int steps, double* dJdgamma_dev) {
  return backward_impl(c, J_seed, steps, dJdgamma_dev, false);
}

// fields of the adjoint state (LKS_FIELD_ADJ_*)
static bool adjoint_field(int which) {
  return which == LKS_FIELD_ADJ_RHO || which == LKS_FIELD_ADJ_VX || which == LKS_FIELD_ADJ_VY ||
         which == LKS_FIELD_ADJ_THETA || which == LKS_FIELD_ADJ_VZ;
}

lks_status lks_read_field(lks_ctx* c, int which, double* dev_out) {
  if (!c || !dev_out) return LKS_E_INVALID;
  if (c->lo && adjoint_field(which)) {
    lks_status st = lks_read_field(c->lo, which, dev_out);
    return st == LKS_OK ? st : fail(c, st, c->lo->err);
  }
  if (!c->bound) return fail(c, LKS_E_STATE, unbound_reason(c));
  lks_status st = c->rsz == 8 ? Run<double>(c).read(which, dev_out)
                              : Run<float>(c).read(which, dev_out);
  if (st != LKS_OK) return fail(c, st, "field not available");
  return check_launch(c);
}

lks_status lks_write_field(lks_ctx* c, int which, const double* dev_in) {
  if (!c || !dev_in) return LKS_E_INVALID;
  if (c->lo && adjoint_field(which)) {
    lks_status st = lks_write_field(c->lo, which, dev_in);
    if (st != LKS_OK) return fail(c, st, c->lo->err);
    c->have_adjoint = true;
    return LKS_OK;
  }
  if (!c->bound) return fail(c, LKS_E_STATE, unbound_reason(c));
  lks_status st = c->rsz == 8 ? Run<double>(c).write(which, dev_in)
                              : Run<float>(c).write(which, dev_in);
  if (st != LKS_OK) return fail(c, st, "field not writable");
  if (which <= LKS_FIELD_T || which == LKS_FIELD_UZ) c->have_forward = true;
  else c->have_adjoint = true;
  return check_launch(c);
}

lks_status lks_set_tile_rows(lks_ctx* c, int tile_rows) {
  if (!c) return LKS_E_INVALID;
  if (c->lo) {
    lks_status st = lks_set_tile_rows(c->lo, tile_rows);
    if (st != LKS_OK) return fail(c, st, c->lo->err);
  }
  if (c->dim == 3) return fail(c, LKS_E_UNSUPPORTED, "D3Q19 kernels are not tiled");
  for (int ty : TILE_ROWS)
    if (ty == tile_rows && tile_rows_ok(ty, c->rsz, c->phys.thermal)) {
      set_tile_rows(c->geo, ty);
      c->have_forward = false;
      c->have_adjoint = false;
      return LKS_OK;
    }
  return fail(c, LKS_E_INVALID, "tile height must be 4 or 8 (or 16 for FP32 non-thermal)");
}

lks_status lks_set_steps_per_launch(lks_ctx* c, int forward_steps, int adjoint_steps) {
  if (!c) return LKS_E_INVALID;
  if (c->lo) {
    // mixed: the forward runs in FP64, the adjoint in FP32
    lks_status st = lks_set_steps_per_launch(c->lo, 1, adjoint_steps);
    if (st != LKS_OK) return fail(c, st, c->lo->err);
    lks_ctx* lo = c->lo;
    c->lo = nullptr;
    st = lks_set_steps_per_launch(c, forward_steps, 1);
    c->lo = lo;
    return st;
  }
  for (int s : {forward_steps, adjoint_steps}) {
    if (s != 1 && s != 2) return fail(c, LKS_E_INVALID, "steps per launch must be 1 or 2");
    if (s == 2 && c->dim != 2)
      return fail(c, LKS_E_UNSUPPORTED, "two steps per launch need a D2Q9 problem");
  }
  if (c->rsz == 8 && ((forward_steps == 2 && c->phys.thermal) || adjoint_steps == 2))
    return fail(c, LKS_E_UNSUPPORTED,
                "FP64 sweeps run two steps per launch for the non-thermal forward only");
  c->spl_f = forward_steps;
  c->spl_a = adjoint_steps;
  return LKS_OK;
}

lks_status lks_set_fused_adjoint(lks_ctx* c, int fused) {
  if (!c) return LKS_E_INVALID;
  if (c->dim != 3) return fail(c, LKS_E_UNSUPPORTED, "the fused ALKS step is a D3Q19 kernel");
  if (fused != 0 && fused != 1) return fail(c, LKS_E_INVALID, "fused must be 0 or 1");
  c->geo3.fused = fused;
  return LKS_OK;
}

lks_status lks_set_adjoint_mode(lks_ctx* c, int mode) {
  if (!c) return LKS_E_INVALID;
  if (mode != LKS_ADJ_PAPER && mode != LKS_ADJ_EXACT)
    return fail(c, LKS_E_INVALID, "adjoint mode must be LKS_ADJ_PAPER or LKS_ADJ_EXACT");
  if (mode != c->adj_exact) c->have_adjoint = false;
  c->adj_exact = mode;
  if (c->lo) return lks_set_adjoint_mode(c->lo, mode);
  return LKS_OK;
}

lks_status lks_set_checkpointing(lks_ctx* c, int scheme, int slots) {
  if (!c) return LKS_E_INVALID;
  if (c->bound) return fail(c, LKS_E_STATE, "checkpointing is planned before lks_bind_workspace");
  if (c->mode != LKS_UNSTEADY)
    return fail(c, LKS_E_UNSUPPORTED, "checkpointing applies to unsteady problems");
  if (scheme != LKS_CKPT_AUTO && scheme != LKS_CKPT_TWO_LEVEL && scheme != LKS_CKPT_BINOMIAL)
    return fail(c, LKS_E_INVALID, "unknown checkpointing scheme");
  if (slots < 0 || (slots > 0 && scheme != LKS_CKPT_BINOMIAL))
    return fail(c, LKS_E_INVALID, "slots must be >= 0, and 0 unless the scheme is binomial");
  const int old_scheme = c->ckpt_scheme, old_slots = c->ckpt_slots;
  c->ckpt_scheme = scheme;
  c->ckpt_slots = slots;
  lks_status st = plan_memory(c);
  if (st != LKS_OK) {
    c->err = g_create_error;
    c->ckpt_scheme = old_scheme;
    c->ckpt_slots = old_slots;
    plan_memory(c);
  }
  return st;
}

lks_status lks_checkpoint_info(const lks_ctx* c, int* scheme, int* count, long long* replay_steps) {
  if (!c) return LKS_E_INVALID;
  const bool uns = c->mode == LKS_UNSTEADY;
  if (scheme) *scheme = uns ? c->plan.scheme : 0;
  if (count)
    *count = !uns ? 0 : (c->plan.scheme == LKS_CKPT_BINOMIAL ? c->plan.n_ckpt
                                                             : std::min(c->plan.K, c->n_steps));
  if (replay_steps) *replay_steps = uns ? c->plan.replay : 0;
  return LKS_OK;
}

lks_status lks_launch_shape(const lks_ctx* c, int* tile_rows, int* forward_steps,
                            int* adjoint_steps) {
  if (!c) return LKS_E_INVALID;
  if (tile_rows) *tile_rows = c->dim == 2 ? c->geo.ty : 0;
  if (forward_steps) *forward_steps = c->spl_f;
  if (adjoint_steps) *adjoint_steps = c->lo ? c->lo->spl_a : c->spl_a;
  return LKS_OK;
}

lks_status lks_autotune(lks_ctx* c, const double* gamma_dev, int steps, int* tile_rows) {
  if (!c || !gamma_dev || steps < 1) return LKS_E_INVALID;
  if (c->lo) {
    // mixed: each part keeps the launch shape that is fastest for its own
    // precision (the FP32 part's forward sweep only serves the timing)
    lks_status st = lks_autotune(c->lo, gamma_dev, steps, nullptr);
    if (st != LKS_OK) return fail(c, st, c->lo->err);
    lks_ctx* lo = c->lo;
    c->lo = nullptr;
    st = lks_autotune(c, gamma_dev, steps, tile_rows);
    c->lo = lo;
    return st;
  }
  if (c->dim == 3) return fail(c, LKS_E_UNSUPPORTED, "D3Q19 kernels are not tiled");
  if (!c->bound) return fail(c, LKS_E_STATE, unbound_reason(c));
  lks_status st = LKS_OK;
  hipEvent_t e[3];
  for (auto& ev : e)
    if (!hip_ok(c, hipEventCreate(&ev), "event", &st)) return st;
  // per tile height, the forward and adjoint sweeps with one and (where
  // supported) two steps per launch, timed separately
  float best = 0.0f;
  int best_ty = c->geo.ty, best_f = c->spl_f, best_a = c->spl_a;
  const int mode = c->mode;
  // two steps per launch exist for FP32 sweeps and the FP64 non-thermal
  // forward; an unsteady adjoint sweep runs one step per launch
  const bool fwd2 = c->rsz == 4 || !c->phys.thermal;
  const int nspl = fwd2 ? 2 : 1;
  c->mode = LKS_STEADY;  // time plain steps on the ping-pong buffers
  for (int ty : TILE_ROWS) {
    if (!tile_rows_ok(ty, c->rsz, c->phys.thermal)) continue;
    set_tile_rows(c->geo, ty);
    float tf[2] = {0.0f, 0.0f}, ta[2] = {0.0f, 0.0f};
    const int nspl_ty = ty == 16 ? 1 : nspl;
    for (int spl = 1; spl <= nspl_ty && st == LKS_OK; ++spl) {
      c->spl_f = c->spl_a = spl;
      for (int rep = 0; rep < 2; ++rep) {  // the first repetition warms up
        hipEventRecord(e[0], c->stream);
        if (c->rsz == 8) {
          Run<double> r(c);
          r.forward(gamma_dev, steps);
          hipEventRecord(e[1], c->stream);
          r.adjoint_steady(1.0, steps, nullptr, true);
        } else {
          Run<float> r(c);
          r.forward(gamma_dev, steps);
          hipEventRecord(e[1], c->stream);
          r.adjoint_steady(1.0, steps, nullptr, true);
        }
        hipEventRecord(e[2], c->stream);
        if (!hip_ok(c, hipEventSynchronize(e[2]), "autotune sync", &st)) break;
        hipEventElapsedTime(&tf[spl - 1], e[0], e[1]);
        hipEventElapsedTime(&ta[spl - 1], e[1], e[2]);
      }
    }
    if (st != LKS_OK) break;
    const int sf = (nspl_ty == 2 && tf[1] < tf[0]) ? 2 : 1;
    const int sa = (nspl_ty == 2 && c->rsz == 4 && mode != LKS_UNSTEADY && ta[1] < ta[0]) ? 2 : 1;
    const float t = tf[sf - 1] + ta[sa - 1];
    if (best == 0.0f || t < best) {
      best = t;
      best_ty = ty;
      best_f = sf;
      best_a = sa;
    }
  }
  c->mode = mode;
  for (auto& ev : e) hipEventDestroy(ev);
  set_tile_rows(c->geo, best_ty);
  c->spl_f = best_f;
  c->spl_a = best_a;
  c->have_forward = false;
  c->have_adjoint = false;
  c->last_level = 0;
  if (tile_rows) *tile_rows = best_ty;
  if (st != LKS_OK) return st;
  return check_launch(c);
}

lks_status lks_memory_report(const lks_ctx* c, size_t* ckpt_bytes, size_t* state_bytes, int* K) {
  if (!c) return LKS_E_INVALID;
  if (ckpt_bytes) *ckpt_bytes = c->plan.ckpt_bytes;
  if (state_bytes) *state_bytes = ws_total(c) - c->plan.ckpt_bytes;
  if (K) *K = c->mode == LKS_UNSTEADY ? std::min(c->plan.K, c->n_steps) : 0;
  return LKS_OK;
}

const char* lks_strerror(lks_status s) {
  switch (s) {
    case LKS_OK: return "ok";
    case LKS_E_INVALID: return "invalid argument";
    case LKS_E_NOMEM: return "not enough memory";
    case LKS_E_HIP: return "HIP runtime error";
    case LKS_E_STATE: return "call out of order";
    case LKS_E_DIVERGED: return "state diverged";
    case LKS_E_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* lks_last_error(const lks_ctx* c) {
  return c ? c->err.c_str() : g_create_error.c_str();
}

void lks_destroy(lks_ctx* c) {
  if (c && c->lo) lks_destroy(c->lo);
  if (c && c->static_dev >= 0) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch.find(c->static_dev);
    if (it != g_scratch.end() && it->second.owner == c) it->second.owner = nullptr;
  }
  delete c;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batches: many independent steady designs, one launch per step
// ---------------------------------------------------------------------------
struct lks_batch {
  int n = 0;
  std::vector<lks_ctx*> ctx;
  std::vector<size_t> off;  // workspace offset of each design's slice
  int rsz = 4;
  int thermal = 0;
  int ty = 8;
  hipStream_t user = nullptr;
  hipStream_t own = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  size_t total = 0;
  bool bound = false;
  char* ws = nullptr;
  std::vector<int> tile0;
  int total_tiles = 0;
  int max_tiles = 0;        // tiles of all designs at the shortest tile height
  std::vector<int> tmap;    // (design, tile within the design) of every global tile
  // device
  int* d_tmap = nullptr;
  void* d_fwd = nullptr;     // BatchFwd<R>[n]
  void* d_adj = nullptr;     // BatchAdj<R>[3 n]: parities 0, 1 and the zero-input first step
  double* d_J = nullptr;
  double* d_sens = nullptr;  // n * maxN doubles
  void* d_zero = nullptr;    // maxN values, all zero
  size_t maxN = 0;
  // graph of the last (n_fwd, n_adj)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int g_nf = -1, g_na = -1;
  int last_nf = 0, last_na = 0;
  bool have_run = false;
  // unsteady batches: checkpointed sweeps over the horizon n_steps shared by
  // the designs, with one checkpoint interval K for all of them
  int unsteady = 0;
  int n_steps = 0;
  int K = 0;
  size_t budget = 0;        // device bytes of the whole batch (0: no limit)
  void* d_store = nullptr;  // BatchStore<R>[n]
  int exact = 0;            // adjoint mode (LKS_ADJ_*)
  std::string err;
};

namespace {

lks_status bfail(lks_batch* b, lks_status s, const std::string& msg) {
  if (b) b->err = msg;
  else g_create_error = msg;
  return s;
}

// (design, tile within the design) of every global tile at the current tile
// height: the batched kernels look their tile up with one load
void build_tile_map(lks_batch* b) {
  b->tmap.assign(2 * size_t(b->total_tiles), 0);
  for (int d = 0; d < b->n; ++d) {
    const int nt = n_tiles(b->ctx[d]->geo);
    for (int t = 0; t < nt; ++t) {
      b->tmap[2 * size_t(b->tile0[d] + t)] = d;
      b->tmap[2 * size_t(b->tile0[d] + t) + 1] = t;
    }
  }
}

// workspace slices of the designs, then the batch's own tables
void batch_layout(lks_batch* b) {
  size_t off = 0;
  b->off.clear();
  for (auto* c : b->ctx) {
    b->off.push_back(off);
    off += align256(c->plan.total);
  }
  const size_t fwd = sizeof(lks::BatchFwd<double>) * b->n;  // the double variants are larger
  const size_t adj = sizeof(lks::BatchAdj<double>) * 3 * b->n;
  off += align256(sizeof(int) * 2 * size_t(b->max_tiles)) + align256(fwd) + align256(adj) +
         align256(sizeof(double) * b->n);
  off += align256(sizeof(double) * b->maxN * b->n) + align256(size_t(b->rsz) * b->maxN);
  off += align256(sizeof(lks::BatchStore<double>) * b->n);
  b->total = off;
}

// unsteady batches: the checkpoint interval shared by the designs, the one
// that replays the fewest steps with the whole batch within the budget (of
// equal replay counts the one that needs the least memory), as one design's
// two-level plan is chosen
lks_status plan_batch(lks_batch* b) {
  const int n = b->n_steps;
  int best = 0;
  long long best_rep = 0;
  size_t best_t = 0, smallest = ~size_t(0);
  for (int K = 1; K <= n + 1; ++K) {
    for (auto* c : b->ctx) set_two_level(c, K);
    batch_layout(b);
    smallest = std::min(smallest, b->total);
    if (b->budget != 0 && b->total > b->budget) continue;
    const long long ls = (long long)(n / K) * K;
    const long long rep = K > n ? 0 : ls - ls / K;
    if (best == 0 || rep < best_rep || (rep == best_rep && b->total < best_t)) {
      best = K;
      best_rep = rep;
      best_t = b->total;
    }
  }
  const int K = best ? best : (b->K ? b->K : n + 1);
  for (auto* c : b->ctx) set_two_level(c, K);
  batch_layout(b);
  if (!best) {
    char buf[160];
    snprintf(buf, sizeof buf, "memory budget %zu B below the smallest checkpoint plan (%zu B)",
             b->budget, smallest);
    return bfail(b, LKS_E_NOMEM, buf);
  }
  b->K = best;
  return LKS_OK;
}

// place of level n when the levels above `base` are held in the replay
// slots (the forward sweep: base = the last checkpoint level), as
// Run::level lays them out
lks::LevelRef level_ref(int n, int base, int K) {
  if (n % K == 0) return {lks::LVL_CKPT, n / K, n & 1};
  if (n > base) return {lks::LVL_SLOT, n - base - 1, n & 1};
  return {lks::LVL_PING, 0, n & 1};
}

template <typename R>
void build_batch_desc(lks_batch* b, double seed, int nf, std::vector<char>& fwd,
                      std::vector<char>& adj) {
  fwd.assign(sizeof(lks::BatchFwd<R>) * b->n, 0);
  adj.assign(sizeof(lks::BatchAdj<R>) * 3 * b->n, 0);
  auto* F = reinterpret_cast<lks::BatchFwd<R>*>(fwd.data());
  auto* Aj = reinterpret_cast<lks::BatchAdj<R>*>(adj.data());
  for (int d = 0; d < b->n; ++d) {
    lks_ctx* c = b->ctx[d];
    F[d].g = c->geo;
    for (int p = 0; p < 2; ++p) {
      lks::FwdArgs<R>& a = F[d].a[p];
      a.mask = c->d_mask;
      a.inv1pa = rp<R>(c->inv1pa);
      a.B = rp<R>(c->B);
      a.ubx = rp<R>(c->ubx);
      a.uby = rp<R>(c->uby);
      a.Tb = rp<R>(c->Tb);
      a.ufac = c->d_ufac;
      a.level_out = 0;
      a.d0 = rp<R>(c->S[p][0]);
      a.ux0 = rp<R>(c->S[p][1]);
      a.uy0 = rp<R>(c->S[p][2]);
      a.T0 = rp<R>(c->S[p][3]);
      a.d1 = rp<R>(c->S[p ^ 1][0]);
      a.ux1 = rp<R>(c->S[p ^ 1][1]);
      a.uy1 = rp<R>(c->S[p ^ 1][2]);
      a.T1 = rp<R>(c->S[p ^ 1][3]);
      a.acc = b->unsteady ? c->acc : nullptr;
      a.objective = c->objective;
    }
    const int fin = nf & 1;  // ping-pong index of the final forward level
    for (int v = 0; v < 3; ++v) {
      lks::BatchAdj<R>& D = Aj[v * b->n + d];
      D.g = c->geo;
      for (int p = 0; p < 2; ++p) {
        lks::AdjArgs<R>& a = D.a[p];
        a.mask = c->d_mask;
        a.inv1pa = rp<R>(c->inv1pa);
        a.B = rp<R>(c->B);
        a.dA3 = rp<R>(c->dA3);
        a.dB = rp<R>(c->dB);
        a.ux = rp<R>(c->S[fin][1]);
        a.uy = rp<R>(c->S[fin][2]);
        a.T = rp<R>(c->S[fin][3]);
        const bool zero = v == 2;
        const R* z = rp<R>(b->d_zero);
        a.r0 = zero ? z : rp<R>(c->P[p][0]);
        a.vx0 = zero ? z : rp<R>(c->P[p][1]);
        a.vy0 = zero ? z : rp<R>(c->P[p][2]);
        a.th0 = zero ? z : rp<R>(c->P[p][3]);
        a.r1 = rp<R>(c->P[p ^ 1][0]);
        a.vx1 = rp<R>(c->P[p ^ 1][1]);
        a.vy1 = rp<R>(c->P[p ^ 1][2]);
        a.th1 = rp<R>(c->P[p ^ 1][3]);
        a.ops = static_cast<const lks::RingOpT<R>*>(c->d_ops);
        a.sens = b->d_sens + size_t(d) * b->maxN;
        a.sens_mode = 0;
        a.exact = b->exact;
        // unsteady: the weight of one level of the time average
        const double w = b->unsteady ? seed / b->n_steps : seed;
        a.seed_dp = c->objective == LKS_OBJ_PRESSURE_DROP ? w : 0.0;
        a.seed_heat = c->objective == LKS_OBJ_HEAT ? w : 0.0;
      }
    }
  }
}

template <typename R>
void build_batch_store(lks_batch* b, std::vector<char>& out) {
  out.assign(sizeof(lks::BatchStore<R>) * b->n, 0);
  auto* S = reinterpret_cast<lks::BatchStore<R>*>(out.data());
  for (int d = 0; d < b->n; ++d) {
    lks_ctx* c = b->ctx[d];
    S[d].C = rp<R>(c->C);
    S[d].Seg = rp<R>(c->Seg);
    for (int p = 0; p < 2; ++p)
      for (int f = 0; f < 4; ++f) S[d].S[p][f] = rp<R>(c->S[p][f]);
    S[d].N = c->N;
    S[d].ckf = ckpt_fields(c);
    S[d].slf = slot_fields(c);
    S[d].n_ufac = int(c->ufac.size());
  }
}

// the step sequence of one batch run: n_fwd LKS steps of every design, the
// pressure drop of every design, n_adj ALKS steps with the last writing the
// sensitivity
template <typename R>
void enqueue_batch_steps(lks_batch* b, int nf, int na, hipStream_t s) {
  auto* F = static_cast<const lks::BatchFwd<R>*>(b->d_fwd);
  auto* Aj = static_cast<const lks::BatchAdj<R>*>(b->d_adj);
  for (int k = 0; k < nf; ++k)
    lks::launch_lks_step_batch<R>(F, b->d_tmap, b->total_tiles, b->ty, b->thermal, k & 1, s);
  lks::launch_pressure_drop_batch<R>(F, b->n, nf & 1, b->d_J, s);
  for (int k = 0; k < na; ++k) {
    const lks::BatchAdj<R>* D = k == 0 ? Aj + 2 * b->n : Aj;
    lks::launch_alks_step_batch<R>(D, b->d_tmap, b->total_tiles, b->ty, b->thermal, k & 1,
                                   k == na - 1, s);
  }
}

// the checkpointed sweeps of an unsteady batch, Run::forward and
// Run::adjoint_unsteady for every design at once: N LKS steps with the
// objective accumulated per tile, the objective sums, then per segment from
// the last down the replay of its levels and its ALKS steps (the first one
// from the zero terminal condition), the sensitivity summed over levels
template <typename R>
void enqueue_batch_unsteady(lks_batch* b, bool adjoint, hipStream_t s) {
  auto* F = static_cast<const lks::BatchFwd<R>*>(b->d_fwd);
  auto* Aj = static_cast<const lks::BatchAdj<R>*>(b->d_adj);
  auto* St = static_cast<const lks::BatchStore<R>*>(b->d_store);
  const int N = b->n_steps, K = b->K, ls = (N / K) * K;
  const bool th = b->thermal;
  lks::launch_acc_zero_batch<R>(F, b->n, s);
  for (int n = 0; n < N; ++n)
    lks::launch_lks_step_ubatch<R>(F, St, b->d_tmap, b->total_tiles, b->ty, th,
                                   level_ref(n, ls, K), level_ref(n + 1, ls, K), n + 1, 1, s);
  lks::launch_acc_sum_batch<R>(F, b->n, b->d_J, s);
  if (!adjoint) return;
  lks::launch_fill(b->d_sens, b->maxN * size_t(b->n), 0.0, s);
  int par = 0;
  for (int base = ls; base >= 0; base -= K) {
    const int top = base == ls ? N : base + K - 1;
    if (base != ls)
      for (int n = base; n < top; ++n)
        lks::launch_lks_step_ubatch<R>(F, St, b->d_tmap, b->total_tiles, b->ty, th,
                                       level_ref(n, base, K), level_ref(n + 1, base, K), n + 1,
                                       0, s);
    for (int n = top; n >= base; --n) {
      const lks::BatchAdj<R>* D = (base == ls && n == top) ? Aj + 2 * b->n : Aj;
      lks::launch_alks_step_ubatch<R>(D, St, b->d_tmap, b->total_tiles, b->ty, th, par,
                                      level_ref(n, base, K), n >= 1 ? 1 : 0,
                                      (n == 0 && b->exact) ? 1 : 0, s);
      par ^= 1;
    }
  }
}

void enqueue_batch(lks_batch* b, int nf, int na, hipStream_t s) {
  if (b->unsteady) {
    if (b->rsz == 8) enqueue_batch_unsteady<double>(b, na > 0, s);
    else enqueue_batch_unsteady<float>(b, na > 0, s);
  } else {
    if (b->rsz == 8) enqueue_batch_steps<double>(b, nf, na, s);
    else enqueue_batch_steps<float>(b, nf, na, s);
  }
}

}  // namespace

static lks_status batch_set_tile_rows(lks_batch* b, int ty);

extern "C" {

lks_status lks_batch_create(int n, const lks_grid* grids, const lks_phys* phys, const lks_bc* bcs,
                            void* hip_stream, lks_batch** out) {
  if (!out) return bfail(nullptr, LKS_E_INVALID, "null output pointer");
  *out = nullptr;
  if (n < 1 || !grids || !phys || !bcs) return bfail(nullptr, LKS_E_INVALID, "empty batch");
  lks_batch* b = new lks_batch();
  b->n = n;
  b->user = static_cast<hipStream_t>(hip_stream);
  b->unsteady = bcs[0].mode == LKS_UNSTEADY ? 1 : 0;
  b->n_steps = b->unsteady ? bcs[0].n_steps : 0;
  for (int d = 0; d < n; ++d) {
    const bool steady_ok = bcs[d].mode == LKS_STEADY && bcs[d].objective == LKS_OBJ_PRESSURE_DROP;
    const bool unsteady_ok =
        bcs[d].mode == LKS_UNSTEADY &&
        (bcs[d].objective == LKS_OBJ_PRESSURE_DROP || bcs[d].objective == LKS_OBJ_HEAT);
    if (!(steady_ok || unsteady_ok) || grids[d].lattice != LKS_D2Q9 ||
        grids[d].precision == LKS_MIXED || phys[d].beta_max > 0.0) {
      for (auto* p : b->ctx) lks_destroy(p);
      delete b;
      return bfail(nullptr, LKS_E_UNSUPPORTED,
                   "batches hold D2Q9 problems without a heat source: steady with the "
                   "pressure-drop objective, or unsteady with the pressure-drop or "
                   "enthalpy-flux objective");
    }
    if (grids[d].precision != grids[0].precision || phys[d].thermal != phys[0].thermal ||
        bcs[d].mode != bcs[0].mode || (b->unsteady && bcs[d].n_steps != b->n_steps)) {
      for (auto* p : b->ctx) lks_destroy(p);
      delete b;
      return bfail(nullptr, LKS_E_INVALID,
                   "designs of a batch share precision, physics kind, mode and (unsteady) "
                   "the horizon n_steps");
    }
    lks_ctx* c = nullptr;
    lks_status st = lks_create(&grids[d], &phys[d], &bcs[d], 0, hip_stream, &c);
    if (st != LKS_OK) {
      for (auto* p : b->ctx) lks_destroy(p);
      delete b;
      return bfail(nullptr, st, "design " + std::to_string(d) + ": " + g_create_error);
    }
    b->ctx.push_back(c);
    b->tile0.push_back(b->total_tiles);
    b->total_tiles += n_tiles(c->geo);
    b->max_tiles += max_tiles(c->geo);
    b->maxN = std::max(b->maxN, size_t(c->geo.N));
    b->ty = c->geo.ty;
  }
  b->rsz = b->ctx[0]->rsz;
  b->thermal = phys[0].thermal ? 1 : 0;
  if (b->unsteady) {
    // tile heights of the unsteady step launches: 4 and 8
    if (b->ty == 16) batch_set_tile_rows(b, 8);
    lks_status st = plan_batch(b);  // no budget yet: every level kept
    if (st != LKS_OK) {
      g_create_error = b->err;
      lks_batch_destroy(b);
      return st;
    }
  } else {
    batch_layout(b);
  }
  *out = b;
  return LKS_OK;
}

lks_status lks_batch_set_memory_budget(lks_batch* b, size_t bytes) {
  if (!b) return LKS_E_INVALID;
  if (b->bound) return bfail(b, LKS_E_STATE, "the budget is planned before lks_batch_bind_workspace");
  const size_t old = b->budget;
  b->budget = bytes;
  if (!b->unsteady) {
    if (bytes != 0 && b->total > bytes) {
      b->budget = old;
      return bfail(b, LKS_E_NOMEM, "the batch's workspace exceeds the budget");
    }
    return LKS_OK;
  }
  lks_status st = plan_batch(b);
  if (st != LKS_OK) {
    const std::string msg = b->err;
    b->budget = old;
    plan_batch(b);
    return bfail(b, st, msg);
  }
  return LKS_OK;
}

lks_status lks_batch_set_adjoint_mode(lks_batch* b, int mode) {
  if (!b) return LKS_E_INVALID;
  if (mode != LKS_ADJ_PAPER && mode != LKS_ADJ_EXACT)
    return bfail(b, LKS_E_INVALID, "adjoint mode must be LKS_ADJ_PAPER or LKS_ADJ_EXACT");
  if (mode != b->exact) b->have_run = false;
  b->exact = mode;
  for (auto* c : b->ctx) c->adj_exact = mode;
  return LKS_OK;
}

lks_status lks_batch_checkpoint_info(const lks_batch* b, int* K, long long* replay_steps,
                                     size_t* workspace_bytes) {
  if (!b) return LKS_E_INVALID;
  if (K) *K = b->unsteady ? b->K : 0;
  if (replay_steps) *replay_steps = b->unsteady ? b->ctx[0]->plan.replay : 0;
  if (workspace_bytes) *workspace_bytes = b->total;
  return LKS_OK;
}

lks_status lks_batch_workspace_size(const lks_batch* b, size_t* bytes) {
  if (!b || !bytes) return LKS_E_INVALID;
  *bytes = b->total;
  return LKS_OK;
}

lks_status lks_batch_bind_workspace(lks_batch* b, void* dev_ptr, size_t bytes) {
  if (!b) return LKS_E_INVALID;
  if (!dev_ptr || (reinterpret_cast<uintptr_t>(dev_ptr) & 255))
    return bfail(b, LKS_E_INVALID, "workspace must be non-null and 256-byte aligned");
  if (bytes < b->total) return bfail(b, LKS_E_NOMEM, "workspace smaller than lks_batch_workspace_size");
  char* base = static_cast<char*>(dev_ptr);
  for (int d = 0; d < b->n; ++d) {
    lks_status st = lks_bind_workspace(b->ctx[d], base + b->off[d], b->ctx[d]->plan.total);
    if (st != LKS_OK) return bfail(b, st, "design " + std::to_string(d) + ": " + b->ctx[d]->err);
  }
  char* p = base + (b->off.back() + align256(b->ctx.back()->plan.total));
  auto take = [&](size_t s) {
    char* q = p;
    p += align256(s);
    return q;
  };
  b->d_tmap = reinterpret_cast<int*>(take(sizeof(int) * 2 * size_t(b->max_tiles)));
  b->d_fwd = take(sizeof(lks::BatchFwd<double>) * b->n);
  b->d_adj = take(sizeof(lks::BatchAdj<double>) * 3 * b->n);
  b->d_J = reinterpret_cast<double*>(take(sizeof(double) * b->n));
  b->d_sens = reinterpret_cast<double*>(take(sizeof(double) * b->maxN * b->n));
  b->d_zero = take(size_t(b->rsz) * b->maxN);
  b->d_store = take(sizeof(lks::BatchStore<double>) * b->n);
  lks_status st = LKS_OK;
  hipStream_t s = b->user;
  if (b->rsz == 8) lks::launch_fill_r<double>(static_cast<double*>(b->d_zero), b->maxN, s);
  else lks::launch_fill_r<float>(static_cast<float*>(b->d_zero), b->maxN, s);
  build_tile_map(b);
  if (!hip_ok(nullptr, hipMemcpyAsync(b->d_tmap, b->tmap.data(), sizeof(int) * b->tmap.size(),
                                      hipMemcpyHostToDevice, s), "upload tiles", &st) ||
      !hip_ok(nullptr, hipStreamSynchronize(s), "bind sync", &st))
    return bfail(b, st, g_create_error);
  if (!b->own) {
    if (!hip_ok(nullptr, hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking), "stream", &st) ||
        !hip_ok(nullptr, hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming), "event", &st) ||
        !hip_ok(nullptr, hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming), "event", &st))
      return bfail(b, st, g_create_error);
  }
  b->ws = base;
  b->bound = true;
  b->have_run = false;
  return LKS_OK;
}

lks_status lks_batch_run(lks_batch* b, const double* const* gamma_dev, int n_fwd, int n_adj,
                         double J_seed, double* const* dJdgamma_dev, double* J_host,
                         int use_graph) {
  if (!b) return LKS_E_INVALID;
  if (!b->bound) return bfail(b, LKS_E_STATE, "no workspace bound");
  if (!gamma_dev || !dJdgamma_dev || !J_host) return bfail(b, LKS_E_INVALID, "null argument");
  if (b->unsteady) {
    if (n_fwd != b->n_steps) return bfail(b, LKS_E_INVALID, "unsteady batches need n_fwd == n_steps");
    if (n_adj != 0) n_adj = n_fwd;  // the sweep covers every level; 0: no sweep
  } else if (n_fwd < 0 || n_adj < 1) {
    return bfail(b, LKS_E_INVALID, "need n_fwd >= 0 and n_adj >= 1");
  }
  if (!std::isfinite(J_seed)) return bfail(b, LKS_E_INVALID, "seed not finite");
  for (int d = 0; d < b->n; ++d)
    if (!gamma_dev[d] || !dJdgamma_dev[d]) return bfail(b, LKS_E_INVALID, "null design pointer");
  lks_status st = LKS_OK;
  // descriptor tables (host -> device, ordered before the steps)
  std::vector<char> fwd, adj, store;
  if (b->rsz == 8) {
    build_batch_desc<double>(b, J_seed, n_fwd, fwd, adj);
    build_batch_store<double>(b, store);
  } else {
    build_batch_desc<float>(b, J_seed, n_fwd, fwd, adj);
    build_batch_store<float>(b, store);
  }
  hipStream_t s = b->user;
  if (!hip_ok(nullptr, hipMemcpyAsync(b->d_fwd, fwd.data(), fwd.size(), hipMemcpyHostToDevice, s),
              "upload descriptors", &st) ||
      !hip_ok(nullptr, hipMemcpyAsync(b->d_adj, adj.data(), adj.size(), hipMemcpyHostToDevice, s),
              "upload descriptors", &st) ||
      !hip_ok(nullptr, hipMemcpyAsync(b->d_store, store.data(), store.size(),
                                      hipMemcpyHostToDevice, s), "upload descriptors", &st))
    return bfail(b, st, g_create_error);
  // design coefficients and level-0 states
  for (int d = 0; d < b->n; ++d) {
    lks_ctx* c = b->ctx[d];
    c->last_level = 0;
    c->cur = 0;
    // level 0: the ping-pong buffer 0 (steady) or checkpoint 0 (unsteady)
    if (b->rsz == 8) {
      Run<double> r(c);
      r.coefficients(gamma_dev[d]);
      double* s0[5] = {};
      if (b->unsteady) r.level(0, c->plan.ls, s0);
      else for (int f = 0; f < 4; ++f) s0[f] = rp<double>(c->S[0][f]);
      r.init(s0);
    } else {
      Run<float> r(c);
      r.coefficients(gamma_dev[d]);
      float* s0[5] = {};
      if (b->unsteady) r.level(0, c->plan.ls, s0);
      else for (int f = 0; f < 4; ++f) s0[f] = rp<float>(c->S[0][f]);
      r.init(s0);
    }
  }
  if (use_graph) {
    if (b->exec && (b->g_nf != n_fwd || b->g_na != n_adj)) {
      hipGraphExecDestroy(b->exec);
      hipGraphDestroy(b->graph);
      b->exec = nullptr;
      b->graph = nullptr;
    }
    if (!b->exec) {
      if (!hip_ok(nullptr, hipStreamBeginCapture(b->own, hipStreamCaptureModeThreadLocal),
                  "begin capture", &st))
        return bfail(b, st, g_create_error);
      enqueue_batch(b, n_fwd, n_adj, b->own);
      if (!hip_ok(nullptr, hipStreamEndCapture(b->own, &b->graph), "end capture", &st) ||
          !hip_ok(nullptr, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0),
                  "instantiate graph", &st))
        return bfail(b, st, g_create_error);
      b->g_nf = n_fwd;
      b->g_na = n_adj;
    }
    if (!hip_ok(nullptr, hipEventRecord(b->ev_in, s), "event", &st) ||
        !hip_ok(nullptr, hipStreamWaitEvent(b->own, b->ev_in, 0), "wait", &st) ||
        !hip_ok(nullptr, hipGraphLaunch(b->exec, b->own), "graph launch", &st) ||
        !hip_ok(nullptr, hipEventRecord(b->ev_out, b->own), "event", &st) ||
        !hip_ok(nullptr, hipStreamWaitEvent(s, b->ev_out, 0), "wait", &st))
      return bfail(b, st, g_create_error);
  } else {
    enqueue_batch(b, n_fwd, n_adj, s);
  }
  // sensitivities to the caller, objectives to the host
  std::vector<double> Js(b->n);
  for (int d = 0; d < b->n && n_adj > 0; ++d) {
    const size_t N = size_t(b->ctx[d]->geo.N);
    if (!hip_ok(nullptr, hipMemcpyAsync(dJdgamma_dev[d], b->d_sens + size_t(d) * b->maxN,
                                        N * sizeof(double), hipMemcpyDeviceToDevice, s),
                "copy sensitivity", &st))
      return bfail(b, st, g_create_error);
  }
  if (!hip_ok(nullptr, hipMemcpyAsync(Js.data(), b->d_J, sizeof(double) * b->n,
                                      hipMemcpyDeviceToHost, s), "read objectives", &st) ||
      !hip_ok(nullptr, hipStreamSynchronize(s), "batch sync", &st) ||
      !hip_ok(nullptr, hipGetLastError(), "batch launch", &st))
    return bfail(b, st, g_create_error);
  for (int d = 0; d < b->n; ++d) {
    lks_ctx* c = b->ctx[d];
    // the objective as lks_objective forms it from the per-level sums
    const double sj = b->unsteady ? Js[d] / b->n_steps : Js[d];
    if (c->objective == LKS_OBJ_PRESSURE_DROP) J_host[d] = (sj + double(c->n_in - c->n_out)) / 3.0;
    else J_host[d] = sj;
    c->cur = n_fwd & 1;
    c->acur = b->unsteady ? (n_fwd + 1) & 1 : n_adj & 1;
    c->last_level = n_fwd;
    c->have_forward = true;
    c->have_adjoint = n_adj > 0;
  }
  b->last_nf = n_fwd;
  b->last_na = n_adj;
  b->have_run = true;
  return LKS_OK;
}

static lks_status batch_set_tile_rows(lks_batch* b, int ty) {
  b->total_tiles = 0;
  for (int d = 0; d < b->n; ++d) {
    set_tile_rows(b->ctx[d]->geo, ty);
    b->tile0[d] = b->total_tiles;
    b->total_tiles += n_tiles(b->ctx[d]->geo);
  }
  b->ty = ty;
  if (b->exec) {
    hipGraphExecDestroy(b->exec);
    hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
  }
  lks_status st = LKS_OK;
  build_tile_map(b);
  // the upload is ordered before every later launch on the user stream;
  // the host table stays alive with the batch
  if (b->bound &&
      !hip_ok(nullptr, hipMemcpyAsync(b->d_tmap, b->tmap.data(), sizeof(int) * b->tmap.size(),
                                      hipMemcpyHostToDevice, b->user), "upload tiles", &st))
    return bfail(b, st, g_create_error);
  return LKS_OK;
}

lks_status lks_batch_autotune(lks_batch* b, const double* const* gamma_dev, int steps,
                              double* const* scratch_dev, int* tile_rows) {
  if (!b || !gamma_dev || !scratch_dev || steps < 1) return LKS_E_INVALID;
  if (!b->bound) return bfail(b, LKS_E_STATE, "no workspace bound");
  if (b->unsteady)
    return bfail(b, LKS_E_UNSUPPORTED, "unsteady batches take their tile height from lks_batch_set_tile_rows");
  std::vector<double> J(b->n);
  float best = 0.0f;
  int best_ty = b->ty;
  lks_status st = LKS_OK;
  hipEvent_t e0, e1;
  if (!hip_ok(nullptr, hipEventCreate(&e0), "event", &st) ||
      !hip_ok(nullptr, hipEventCreate(&e1), "event", &st))
    return bfail(b, st, g_create_error);
  for (int ty : TILE_ROWS) {
    if (!tile_rows_ok(ty, b->rsz, b->thermal)) continue;
    if ((st = batch_set_tile_rows(b, ty)) != LKS_OK) break;
    float t = 0.0f;
    for (int rep = 0; rep < 2; ++rep) {
      hipEventRecord(e0, b->user);
      st = lks_batch_run(b, gamma_dev, steps, steps, 1.0, scratch_dev, J.data(), 0);
      hipEventRecord(e1, b->user);
      if (st != LKS_OK) break;
      hipEventSynchronize(e1);
      hipEventElapsedTime(&t, e0, e1);
    }
    if (st != LKS_OK) break;
    if (best == 0.0f || t < best) {
      best = t;
      best_ty = ty;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st != LKS_OK) return st;
  if ((st = batch_set_tile_rows(b, best_ty)) != LKS_OK) return st;
  if (tile_rows) *tile_rows = best_ty;
  b->have_run = false;
  return LKS_OK;
}

lks_status lks_batch_set_tile_rows(lks_batch* b, int tile_rows) {
  if (!b) return LKS_E_INVALID;
  bool known = false;
  for (int ty : TILE_ROWS) known = known || ty == tile_rows;
  if (!known || !tile_rows_ok(tile_rows, b->rsz, b->thermal) || (b->unsteady && tile_rows == 16))
    return bfail(b, LKS_E_INVALID,
                 "tile height must be 4 or 8 (or 16 for FP32 non-thermal steady batches)");
  lks_status st = batch_set_tile_rows(b, tile_rows);
  if (st == LKS_OK) b->have_run = false;
  return st;
}

lks_status lks_batch_read_field(lks_batch* b, int design, int which, double* dev_out) {
  if (!b || design < 0 || design >= b->n) return LKS_E_INVALID;
  if (!b->have_run) return bfail(b, LKS_E_STATE, "read before lks_batch_run");
  if (b->unsteady && adjoint_field(which) && b->last_na == 0)
    return bfail(b, LKS_E_STATE, "the last run had no adjoint sweep");
  if (b->unsteady && !adjoint_field(which))
    return bfail(b, LKS_E_UNSUPPORTED,
                 "unsteady batches keep no forward level after the sweep (the replays reuse "
                 "its slots); adjoint fields are those of level 0");
  lks_status st = lks_read_field(b->ctx[design], which, dev_out);
  if (st != LKS_OK) return bfail(b, st, b->ctx[design]->err);
  return LKS_OK;
}

const char* lks_batch_last_error(const lks_batch* b) {
  return b ? b->err.c_str() : g_create_error.c_str();
}

void lks_batch_destroy(lks_batch* b) {
  if (!b) return;
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  if (b->ev_in) hipEventDestroy(b->ev_in);
  if (b->ev_out) hipEventDestroy(b->ev_out);
  if (b->own) hipStreamDestroy(b->own);
  for (auto* c : b->ctx) lks_destroy(c);
  delete b;
}

}  // extern "C"
