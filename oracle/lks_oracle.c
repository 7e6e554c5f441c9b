/*
 * Plain FP64 CPU oracle of the Lattice Kinetic Scheme (LKS) and its adjoint
 * (ALKS) for Brinkman-penalised topology optimisation, after Tanabe, Yaji and
 * Ushijima, "Adjoint lattice kinetic scheme for topology optimization in
 * fluid problems" (arXiv 2411.03090).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, obviously correct
 * definition that the GPU library is checked against. Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never calls it. It shares no code, header, table or constant
 * with the GPU library.
 *
 * Conventions (lattice units, dx = dt = 1, tau_f = tau_g = 1, so the paper's
 * eps_f = eps_g = dx and every (1/eps) dx factor is 1):
 *   - D2Q9, c0=(0,0) c1=(1,0) c2=(0,1) c3=(-1,0) c4=(0,-1) c5=(1,1)
 *     c6=(-1,1) c7=(-1,-1) c8=(1,-1); w = 4/9, 1/9 (x4), 1/36 (x4)
 *     (Sec. 2.3, eq:D2Q9w; the numbering is the one the boundary matrices of
 *     Sec. 2.5 use).
 *   - Fields are node arrays of size nx*ny, x fastest: k = j*nx + i.
 *   - Density is carried as drho = rho - 1. Since sum_i w_i = 1 and
 *     sum_i w_i c_i = 0, the constant part of f_i^eq contributes exactly 1 to
 *     the density and 0 to the momentum, so every sum below is taken over
 *     f'_i = f_i^eq - w_i, which is f_i^eq with drho in place of rho.
 *   - The outer ring of nodes is the boundary; its outward normal follows
 *     from its position. Interior nodes are design nodes.
 *
 * Every function cites the passage of the paper it follows. Readings of
 * passages that are silent or garbled are stated where they are used.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q9 9

static const int CX[Q9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[Q9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W[Q9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

/* node-class byte */
#define FLOW(m) ((m) & 3)
#define FLOW_INTERIOR 0
#define FLOW_VELOCITY 1
#define FLOW_PRESSURE 2
#define FLOW_CORNER 3
#define THERM(m) (((m) >> 2) & 3)
#define THERM_DIRICHLET 1
#define THERM_FLUX 2
#define TAG_J_INLET 16
#define TAG_J_OUTLET 32
#define TAG_PROBE 64

/* objectives */
#define OBJ_HEAT_EXCHANGE 2
#define OBJ_HEAT_SINK 3

typedef struct {
  int nx, ny;
  int periodic;          /* 1: periodic box, every node interior */
  int thermal;           /* 1: temperature field present */
  double nu;             /* kinematic viscosity, eq:A */
  double Kf, Ks, q_K;    /* eq:conductivity */
  double alpha_max, q_alpha; /* eq:brinkman */
  double rho_out;        /* prescribed outlet density (p = rho/3) */
  const uint8_t *mask;   /* nx*ny node classes */
  const double *ubar;    /* 2*nx*ny prescribed velocity (x block, y block) */
  const double *Tbar;    /* nx*ny prescribed temperature; at heat-flux nodes
                            the heat flux qbar into the domain */
  int adj_exact;         /* 1: exact discrete adjoint of the Brinkman step */
  double gbeta[2];       /* g beta of the Boussinesq force eq:boussinesqforce */
  double T_ref;          /* its reference temperature */
  double beta_max, q_beta; /* heat source eq:heatsource with eq:betagamma */
} orc_problem;

/* ------------------------------------------------------------------ */
/* helpers                                                             */
/* ------------------------------------------------------------------ */
static inline int idx(const orc_problem *P, int i, int j) { return j * P->nx + i; }

static inline int on_ring(const orc_problem *P, int i, int j) {
  if (P->periodic) return 0;
  return i == 0 || j == 0 || i == P->nx - 1 || j == P->ny - 1;
}

/* neighbour index of (i,j) shifted by (di,dj); -1 when outside a
 * non-periodic domain */
static inline int nbr(const orc_problem *P, int i, int j, int di, int dj) {
  int a = i + di, b = j + dj;
  if (P->periodic) {
    a = (a % P->nx + P->nx) % P->nx;
    b = (b % P->ny + P->ny) % P->ny;
  } else if (a < 0 || b < 0 || a >= P->nx || b >= P->ny) {
    return -1;
  }
  return idx(P, a, b);
}

/* outward unit normal of a ring node that is not a corner */
static void ring_normal(const orc_problem *P, int i, int j, int *nx_, int *ny_) {
  *nx_ = 0;
  *ny_ = 0;
  if (i == 0) *nx_ = -1;
  else if (i == P->nx - 1) *nx_ = 1;
  else if (j == 0) *ny_ = -1;
  else if (j == P->ny - 1) *ny_ = 1;
}

/* Finite-difference derivative of field f at (i,j) along x (axis 0) or y
 * (axis 1). The paper stores derivative arrays but does not print its
 * stencil; the reading used here: second-order central difference inside,
 * second-order one-sided difference at the two ends of each axis (so along
 * the normal at the boundary and both ways at corners), wrap-around in a
 * periodic box. */
static double ddx(const orc_problem *P, const double *f, int i, int j, int axis) {
  int n = axis == 0 ? P->nx : P->ny;
  int p = axis == 0 ? i : j;
  int sx = axis == 0 ? 1 : 0, sy = axis == 0 ? 0 : 1;
  if (P->periodic || (p > 0 && p < n - 1)) {
    return 0.5 * (f[nbr(P, i, j, sx, sy)] - f[nbr(P, i, j, -sx, -sy)]);
  }
  if (p == 0) {
    return 0.5 * (-3.0 * f[idx(P, i, j)] + 4.0 * f[nbr(P, i, j, sx, sy)] -
                  f[nbr(P, i, j, 2 * sx, 2 * sy)]);
  }
  return 0.5 * (3.0 * f[idx(P, i, j)] - 4.0 * f[nbr(P, i, j, -sx, -sy)] +
                f[nbr(P, i, j, -2 * sx, -2 * sy)]);
}

/* A from the viscosity, eq:A: nu = (1/6 - 2A/9) dx */
static double coef_A(const orc_problem *P) { return 4.5 * (1.0 / 6.0 - P->nu); }

/* ------------------------------------------------------------------ */
/* design -> coefficients                                              */
/* ------------------------------------------------------------------ */
/* eq:brinkman  alpha = abar q (1-g)/(q+g);
 * eq:conductivity K = Kf + (Ks-Kf) qK (1-g)/(qK+g);
 * eq:B  K = (1/6 - B/3) dx  =>  B = 3 (1/6 - K).
 * Boundary-ring nodes are non-design fluid nodes: alpha = 0, B = B(Kf),
 * derivatives 0. */
void orc_coefficients(const orc_problem *P, const double *gamma, double *alpha,
                      double *dalpha, double *B, double *dB) {
  int N = P->nx * P->ny;
  for (int k = 0; k < N; ++k) {
    int i = k % P->nx, j = k / P->nx;
    double g = gamma[k];
    if (on_ring(P, i, j)) {
      alpha[k] = 0.0;
      dalpha[k] = 0.0;
      B[k] = 3.0 * (1.0 / 6.0 - P->Kf);
      dB[k] = 0.0;
      continue;
    }
    double qa = P->q_alpha;
    alpha[k] = P->alpha_max * qa * (1.0 - g) / (qa + g);
    dalpha[k] = -P->alpha_max * qa * (1.0 + qa) / ((qa + g) * (qa + g));
    double qk = P->q_K;
    double K = P->Kf + (P->Ks - P->Kf) * qk * (1.0 - g) / (qk + g);
    double dK = -(P->Ks - P->Kf) * qk * (1.0 + qk) / ((qk + g) * (qk + g));
    B[k] = 3.0 * (1.0 / 6.0 - K);
    dB[k] = -3.0 * dK;
  }
}

/* eq:betagamma  beta = bbar q (1-g)/(q+g), the coefficient of the heat
 * source Q = beta (1 - T) (eq:heatsource) that acts in the solid only.
 * Boundary-ring nodes are non-design: beta = 0, beta' = 0. */
void orc_source_coefficients(const orc_problem *P, const double *gamma,
                             double *beta, double *dbeta) {
  int N = P->nx * P->ny;
  for (int k = 0; k < N; ++k) {
    int i = k % P->nx, j = k / P->nx;
    double g = gamma[k], qb = P->q_beta;
    if (on_ring(P, i, j)) {
      beta[k] = 0.0;
      dbeta[k] = 0.0;
      continue;
    }
    beta[k] = P->beta_max * qb * (1.0 - g) / (qb + g);
    dbeta[k] = -P->beta_max * qb * (1.0 + qb) / ((qb + g) * (qb + g));
  }
}

/* ------------------------------------------------------------------ */
/* forward LKS step                                                    */
/* ------------------------------------------------------------------ */
/* f'_i^eq at node k (eq:feq2 with drho in place of rho):
 * w_i { drho + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u
 *       + A (du_a/dx_b + du_b/dx_a) c_a c_b } */
static double feq(int q, double drho, double ux, double uy, const double G[2][2],
                  double A) {
  double cu = CX[q] * ux + CY[q] * uy;
  double c[2] = {(double)CX[q], (double)CY[q]};
  double strain = 0.0;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) strain += (G[a][b] + G[b][a]) * c[a] * c[b];
  return W[q] * (drho + 3.0 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy) +
                 A * strain);
}

/* g_i^eq at node k, eq:geq2 read as w_i [ T (1 + 3 c.u) + B c.grad T ].
 * The printed form puts T in front of the B term; the linear reading is the
 * one for which eq:B gives a diffusivity independent of T and whose adjoint
 * is the printed eq:ageq (which has no T grad T term). */
static double geq(int q, double T, double ux, double uy, double B, double dTx,
                  double dTy) {
  double cu = CX[q] * ux + CY[q] * uy;
  return W[q] * (T * (1.0 + 3.0 * cu) + B * (CX[q] * dTx + CY[q] * dTy));
}

/* Velocity gradient tensor G[a][b] = du_a/dx_b at (i,j). */
static void vel_grad(const orc_problem *P, const double *ux, const double *uy,
                     int i, int j, double G[2][2]) {
  G[0][0] = ddx(P, ux, i, j, 0);
  G[0][1] = ddx(P, ux, i, j, 1);
  G[1][0] = ddx(P, uy, i, j, 0);
  G[1][1] = ddx(P, uy, i, j, 1);
}

/* Level-0 state: rho = 1, u = 0, T = 0, with the prescribed boundary values
 * (velocity nodes u = ubar * ufac0, temperature nodes T = Tbar) and corners
 * copying the temperature of their neighbour along y. */
void orc_init_state(const orc_problem *P, double ufac0, double *drho, double *ux,
                    double *uy, double *T) {
  int N = P->nx * P->ny;
  for (int k = 0; k < N; ++k) {
    drho[k] = 0.0;
    ux[k] = 0.0;
    uy[k] = 0.0;
    if (T) T[k] = 0.0;
    if (P->periodic) continue;
    uint8_t m = P->mask[k];
    if (FLOW(m) == FLOW_VELOCITY) {
      ux[k] = P->ubar[k] * ufac0;
      uy[k] = P->ubar[N + k] * ufac0;
    }
    if (T && THERM(m) == THERM_DIRICHLET) T[k] = P->Tbar[k];
  }
  if (T && !P->periodic) {
    for (int k = 0; k < N; ++k) {
      if (FLOW(P->mask[k]) != FLOW_CORNER) continue;
      int i = k % P->nx, j = k / P->nx;
      int kn = idx(P, i, j == 0 ? 1 : P->ny - 2);
      T[k] = T[kn];
    }
  }
}

/* One LKS step, level n -> n+1 (eq:lbef2/eq:lbeg2, eq:rho, eq:u, eq:T with
 * eq:feq2, eq:geq2 and the Brinkman force of eq:lbef_ex).
 *
 * Interior: rho = sum_i f_i^eq(x - c_i), U* = sum_i c_i f_i^eq(x - c_i),
 * T = sum_i g_i^eq(x - c_i). The Brinkman term of eq:lbef_ex acts on u at
 * the new level, and its first moment is -alpha u (sum_i 3 w_i c_i c_i = I),
 * so u = U* / (1 + alpha).
 *
 * Boundary nodes (Sec. 2.4 prescribes the macroscopic values; the closures
 * for the values it leaves free are a reading): with outward normal n, the
 * pulled f_i = f_i^eq(x - c_i) are known for c_i.n >= 0. Using
 * rho = sum f_i and u.n = sum (c_i.n) f_i:
 *   velocity node: u = ubar, rho = S0 + 2 S+ - u.n
 *   pressure node: rho = rho_out, u_t = 0, u.n = S0 + 2 S+ - rho_out
 *   heat-flux node: T (1 + u.n) = S0g + 2 S+g + qbar
 *   temperature node: T = Tbar
 * where S0, S+ sum the known f_i with c_i.n = 0 and c_i.n > 0. The heat-flux
 * condition of Sec. 2.4, -q.n = qbar with q = sum c_i g_i - u T (the flux
 * whose variation the kappa~ term of the adjoint boundary conditions
 * carries), fixes the unknown g_i: with S- their sum, S+ - S- - u.n T = -qbar,
 * and T = S0 + S+ + S- gives the closure above (qbar = 0: adiabatic).
 * Corners: u = 0; rho and T copied from the neighbour along y at the new
 * level.
 *
 * Heat source (beta non-NULL): eq:lbeg_ex adds dx w_i Q to g_i (the weight
 * as in the kinetic equation of Appendix A), Q = beta (1 - T) at the new
 * level, so its zeroth moment gives T (1 + beta) = T* + beta. */
void orc_lks_step(const orc_problem *P, const double *alpha, const double *B,
                  const double *beta, double ufac, const double *drho, const double *ux,
                  const double *uy, const double *T, double *drho_o, double *ux_o,
                  double *uy_o, double *T_o) {
  const int nx = P->nx, ny = P->ny, N = nx * ny;
  const double A = coef_A(P);
  const int th = P->thermal;

#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j) {
    for (int i = 0; i < nx; ++i) {
      int k = idx(P, i, j);
      uint8_t m = P->periodic ? 0 : P->mask[k];
      if (FLOW(m) == FLOW_CORNER) continue;
      int nrm[2] = {0, 0};
      int bnd = on_ring(P, i, j);
      if (bnd) ring_normal(P, i, j, &nrm[0], &nrm[1]);

      double rho_s = 0, Ux = 0, Uy = 0, T_s = 0;  /* full pulls (interior) */
      double S0 = 0, Sp = 0, S0g = 0, Spg = 0;    /* partial pulls (ring) */
      for (int q = 0; q < Q9; ++q) {
        int cn = CX[q] * nrm[0] + CY[q] * nrm[1];
        if (bnd && cn < 0) continue; /* would come from outside */
        int kz = nbr(P, i, j, -CX[q], -CY[q]);
        int iz = kz % nx, jz = kz / nx;
        double G[2][2];
        vel_grad(P, ux, uy, iz, jz, G);
        double f = feq(q, drho[kz], ux[kz], uy[kz], G, A);
        double g = 0.0;
        if (th) {
          double dTx = ddx(P, T, iz, jz, 0), dTy = ddx(P, T, iz, jz, 1);
          g = geq(q, T[kz], ux[kz], uy[kz], B[kz], dTx, dTy);
        }
        rho_s += f;
        Ux += CX[q] * f;
        Uy += CY[q] * f;
        T_s += g;
        if (cn == 0) { S0 += f; S0g += g; }
        if (cn > 0) { Sp += f; Spg += g; }
      }

      if (!bnd) {
        /* eq:lbef_ex with the Brinkman and the Boussinesq force
         * G = g beta (T - T_ref) (eq:boussinesqforce) at the new level:
         * u (1 + alpha) = U* + G */
        double Gx = 0.0, Gy = 0.0;
        if (th && beta) T_s = (T_s + beta[k]) / (1.0 + beta[k]);
        if (th) {
          Gx = P->gbeta[0] * (T_s - P->T_ref);
          Gy = P->gbeta[1] * (T_s - P->T_ref);
        }
        drho_o[k] = rho_s;
        ux_o[k] = (Ux + Gx) / (1.0 + alpha[k]);
        uy_o[k] = (Uy + Gy) / (1.0 + alpha[k]);
        if (th) T_o[k] = T_s;
        continue;
      }
      double un;
      if (FLOW(m) == FLOW_VELOCITY) {
        ux_o[k] = P->ubar[k] * ufac;
        uy_o[k] = P->ubar[N + k] * ufac;
        un = ux_o[k] * nrm[0] + uy_o[k] * nrm[1];
        drho_o[k] = S0 + 2.0 * Sp - un;
      } else { /* pressure outlet */
        double drho_out = P->rho_out - 1.0;
        drho_o[k] = drho_out;
        un = S0 + 2.0 * Sp - drho_out;
        ux_o[k] = un * nrm[0];
        uy_o[k] = un * nrm[1];
      }
      if (th) {
        if (THERM(m) == THERM_DIRICHLET) T_o[k] = P->Tbar[k];
        else T_o[k] = (S0g + 2.0 * Spg + P->Tbar[k]) / (1.0 + un);
      }
    }
  }
  if (P->periodic) return;
  /* corners, after their neighbours */
  for (int k = 0; k < N; ++k) {
    if (FLOW(P->mask[k]) != FLOW_CORNER) continue;
    int i = k % nx, j = k / nx;
    int kn = idx(P, i, j == 0 ? 1 : ny - 2);
    drho_o[k] = drho_o[kn];
    ux_o[k] = 0.0;
    uy_o[k] = 0.0;
    if (th) T_o[k] = T_o[kn];
  }
}

/* ------------------------------------------------------------------ */
/* objectives                                                          */
/* ------------------------------------------------------------------ */
/* Static pressure drop eq:objective_pipebend with dGamma = dx = 1 and
 * p = rho/3 (eq:lbmp): sum over inlet nodes minus sum over outlet nodes. */
double orc_pressure_drop(const orc_problem *P, const double *drho) {
  double s = 0.0;
  int N = P->nx * P->ny;
  for (int k = 0; k < N; ++k) {
    if (P->mask[k] & TAG_J_INLET) s += (1.0 + drho[k]) / 3.0;
    if (P->mask[k] & TAG_J_OUTLET) s -= (1.0 + drho[k]) / 3.0;
  }
  return s;
}

/* Enthalpy flux u_x T summed over the probe nodes (the per-level integrand
 * of the heat-transfer objective; its time average is the objective). */
double orc_probe_heat(const orc_problem *P, const double *ux, const double *T) {
  double s = 0.0;
  int N = P->nx * P->ny;
  for (int k = 0; k < N; ++k)
    if (P->mask[k] & TAG_PROBE) s += ux[k] * T[k];
  return s;
}

/* Heat-sink objective eq:objective_heatsink at one level: the mean
 * temperature over the probe-tagged (heated) boundary nodes. */
double orc_probe_T(const orc_problem *P, const double *T) {
  double s = 0.0;
  int n = 0, N = P->nx * P->ny;
  for (int k = 0; k < N; ++k)
    if (P->mask[k] & TAG_PROBE) {
      s += T[k];
      ++n;
    }
  return n ? s / n : 0.0;
}

/* Heat-exchange objective eq:objective_heatexchanger at one level:
 * J = -sum_nodes beta (1 - T) (dOmega = dx^2 = 1). */
double orc_source_heat(const orc_problem *P, const double *beta, const double *T) {
  double s = 0.0;
  int N = P->nx * P->ny;
  for (int k = 0; k < N; ++k) s -= beta[k] * (1.0 - T[k]);
  return s;
}

/* ------------------------------------------------------------------ */
/* adjoint: equilibrium coefficients                                   */
/* ------------------------------------------------------------------ */
/* Adjoint state layout: 9 arrays of nx*ny
 *   0 rho~  1 u~x  2 u~y  3 s~xx  4 s~xy  5 s~yy  6 T~  7 q~x  8 q~y
 * (s~ is symmetric by eq:as, so s~yx = s~xy.) */
enum { A_R = 0, A_UX, A_UY, A_SXX, A_SXY, A_SYY, A_T, A_QX, A_QY, A_NF };

/* eq:afeq: f~_i^eq = rho~ + c_i . V with
 *   V_a = 3 u~_a + 9 s~_ab u_b - 3 rho~ u_a - A d/dx_b (s~_ab + s~_ba)
 * eq:ageq: g~_i^eq = Theta (independent of i) with
 *   Theta = T~ + 3 q~.u - B div q~ - grad B . q~
 * evaluated with the state (u, T) of the same time level. */
static void adj_V(const orc_problem *P, int i, int j, const double *ux,
                  const double *uy, const double *const *adj, double V[2]) {
  const double A = coef_A(P);
  int k = idx(P, i, j);
  double r = adj[A_R][k];
  double u[2] = {ux[k], uy[k]};
  double s[2][2] = {{adj[A_SXX][k], adj[A_SXY][k]}, {adj[A_SXY][k], adj[A_SYY][k]}};
  /* d/dx_b (s~_ab + s~_ba) = 2 d/dx_b s~_ab */
  double divs[2];
  divs[0] = 2.0 * (ddx(P, adj[A_SXX], i, j, 0) + ddx(P, adj[A_SXY], i, j, 1));
  divs[1] = 2.0 * (ddx(P, adj[A_SXY], i, j, 0) + ddx(P, adj[A_SYY], i, j, 1));
  double ut[2] = {adj[A_UX][k], adj[A_UY][k]};
  for (int a = 0; a < 2; ++a)
    V[a] = 3.0 * ut[a] + 9.0 * (s[a][0] * u[0] + s[a][1] * u[1]) - 3.0 * r * u[a] -
           A * divs[a];
}

/* With alpha given (exact mode), V is divided by 1 + alpha at its node: the
 * transpose of u = U* / (1 + alpha) applied where the velocity was formed.
 * With beta given as well (heat source), Theta is divided by 1 + beta at its
 * node in the same way, the transpose of T = (T* + beta) / (1 + beta).
 * The exact mode (the problem's flag, with or without alpha) also takes the
 * transpose of the forward term B c_i.grad_h T:
 * -div_h (B q~), the difference stencil applied to the product, in place of
 * the product rule -B div q~ - grad B . q~ of eq:ageq (the two agree for
 * uniform B; the transpose is exact on periodic grids). */
void orc_adjoint_equilibrium(const orc_problem *P, const double *B,
                             const double *ux, const double *uy,
                             const double *const *adj, double *Vx, double *Vy,
                             double *Theta, const double *alpha,
                             const double *beta) {
  const int nx = P->nx, ny = P->ny, N = nx * ny;
  double *Bq = NULL;
  if (Theta && P->adj_exact) {
    Bq = malloc(2 * (size_t)N * sizeof(double));
    for (int k = 0; k < N; ++k) {
      Bq[k] = B[k] * adj[A_QX][k];
      Bq[N + k] = B[k] * adj[A_QY][k];
    }
  }
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j) {
    for (int i = 0; i < nx; ++i) {
      int k = idx(P, i, j);
      double u[2] = {ux[k], uy[k]};
      double V[2];
      adj_V(P, i, j, ux, uy, adj, V);
      const double sc = alpha ? 1.0 / (1.0 + alpha[k]) : 1.0;
      Vx[k] = V[0] * sc;
      Vy[k] = V[1] * sc;
      if (Theta) {
        double qx = adj[A_QX][k], qy = adj[A_QY][k];
        double divq = ddx(P, adj[A_QX], i, j, 0) + ddx(P, adj[A_QY], i, j, 1);
        double dBx = ddx(P, B, i, j, 0), dBy = ddx(P, B, i, j, 1);
        if (Bq)
          Theta[k] = adj[A_T][k] + 3.0 * (qx * u[0] + qy * u[1]) -
                     (ddx(P, Bq, i, j, 0) + ddx(P, Bq + N, i, j, 1));
        else
          Theta[k] = adj[A_T][k] + 3.0 * (qx * u[0] + qy * u[1]) - B[k] * divq -
                     (dBx * qx + dBy * qy);
        /* exact mode: the propagated Theta also carries the dependence of
         * the new velocity on the new temperature through G, whose adjoint
         * is g beta . V / (1 + alpha) at interior nodes */
        if (alpha && !on_ring(P, i, j))
          Theta[k] += (P->gbeta[0] * V[0] + P->gbeta[1] * V[1]) * sc;
        if (alpha && beta) Theta[k] /= 1.0 + beta[k];
      }
    }
  }
  free(Bq);
}

/* ------------------------------------------------------------------ */
/* small dense least squares                                            */
/* ------------------------------------------------------------------ */
/* Minimise || K x + b ||_2 over x (K is rows x cols, row-major) through the
 * normal equations (K^T K) x = -K^T b, solved by Gaussian elimination with
 * partial pivoting. This is the generalized-inverse solution of Sec. 2.5
 * (the solution minimises the residual norm, eq:r_definition). */
static void lsq_solve(int rows, int cols, const double *K, const double *b,
                      double *x) {
  double G[16][17];
  for (int a = 0; a < cols; ++a) {
    for (int c = 0; c < cols; ++c) {
      double s = 0;
      for (int r = 0; r < rows; ++r) s += K[r * cols + a] * K[r * cols + c];
      G[a][c] = s;
    }
    double h = 0;
    for (int r = 0; r < rows; ++r) h += K[r * cols + a] * b[r];
    G[a][cols] = -h;
  }
  for (int p = 0; p < cols; ++p) {
    int piv = p;
    for (int r = p + 1; r < cols; ++r)
      if (fabs(G[r][p]) > fabs(G[piv][p])) piv = r;
    if (piv != p)
      for (int c = 0; c <= cols; ++c) {
        double t = G[p][c];
        G[p][c] = G[piv][c];
        G[piv][c] = t;
      }
    for (int r = p + 1; r < cols; ++r) {
      double f = G[r][p] / G[p][p];
      for (int c = p; c <= cols; ++c) G[r][c] -= f * G[p][c];
    }
  }
  for (int p = cols - 1; p >= 0; --p) {
    double s = G[p][cols];
    for (int c = p + 1; c < cols; ++c) s -= G[p][c] * x[c];
    x[p] = s / G[p][p];
  }
}

/* Adjoint boundary fill at one ring node (Sec. 2.5 and Appendix A).
 *
 * Flow rows, for every i = 0..8 (velocity node: eq:afboundaryu; pressure
 * node: eq:afboundaryp; flux-thermal nodes add -kappa~ T (c_i.n), from
 * eq:afboundaryuq / eq:afboundarypq):
 *   r_i = (n.c_i) f~_i - 2A sum_j w_j (n.c_j)(c_j.c_i) f~_j
 *         + [mu~.c_i | lambda~ + mu~_s (c_i.t)] - kappa~ T (c_i.n) + s_i
 * where the s~ of the printed condition is expanded through eq:afs. The
 * printed matrix M is garbled (it repeats c_b c_b); this reading is the one
 * that reproduces the printed closed form eq:ftilde, with least squares over
 * all nine rows. Unknowns: f~_i with c_i.n > 0 and the multipliers.
 * s_i = dJ_dO/df_i, the boundary seed. Reading: for the pressure-drop
 * objective (J_dO = p on inlet nodes, -p on outlet nodes) s_i is the
 * derivative of J_dO with respect to the boundary pressure, +seed on inlet
 * nodes and -seed on outlet nodes, in every row. The least-squares solution
 * takes -2 s_i into each unknown, so the completed set carries an adjoint
 * velocity with 3 u~.n = -s_i: the adjoint velocity that the continuous
 * adjoint of a velocity boundary carries for an objective that integrates
 * the pressure there. Taken literally, p = sum f_i / 3 would give seed/3,
 * and with it the gradient of the paper's own non-thermal check (Sec. 2.6,
 * where ALKS and finite differences are reported in strong agreement) comes
 * out uniformly one third of central differences; with the pressure
 * derivative it agrees with them to about 2 %. On outlet nodes the seed is
 * taken up by lambda~ in either reading.
 *
 * Thermal rows (eq:agboundaryT / eq:agboundaryq), for every i:
 *   r_i = (n.c_i) g~_i - B (n.q~) + [eta~ | kappa~ (c_i - u).n] + s_T
 * with q~ expanded through eq:agq and s_T a row seed (every row alike; the
 * heat-sink objective enters the adjoint differently, see orc_alks_step, and
 * passes 0 here). Unknowns: g~_i with c_i.n > 0 and the
 * multiplier. The thermal system does not involve f~, so it is solved first
 * and its kappa~ enters the flow rows as a known term.
 *
 * Inputs: fk[i], gk[i] hold the known (pulled) values for c_i.n <= 0.
 * Outputs: fk, gk completed in place. */
static void boundary_fill(const orc_problem *P, uint8_t m, const int n[2],
                          double A, double Bn, double Tn, double unx,
                          double uny, double seed_dp, double seed_T, double *fk,
                          double *gk, double *mult) {
  double cn[Q9];
  for (int q = 0; q < Q9; ++q) cn[q] = CX[q] * n[0] + CY[q] * n[1];
  int unk[Q9], nu = 0;
  for (int q = 0; q < Q9; ++q)
    if (cn[q] > 0) unk[nu++] = q;

  double kappa = 0.0;
  int flux = P->thermal && THERM(m) == THERM_FLUX;
  if (P->thermal) {
    /* thermal system: cols = nu + 1 */
    int cols = nu + 1;
    double K[Q9 * 8], b[Q9], x[8];
    double u_n = unx * n[0] + uny * n[1];
    for (int r = 0; r < Q9; ++r) {
      /* coefficient of g~_j in row r: delta_rj (n.c_r) - B w_j (n.c_j) */
      double known = 0.0;
      for (int q = 0; q < Q9; ++q) {
        double coef = (q == r ? cn[r] : 0.0) - Bn * W[q] * cn[q];
        if (cn[q] <= 0) known += coef * gk[q];
      }
      for (int a = 0; a < nu; ++a) {
        int q = unk[a];
        K[r * cols + a] = (q == r ? cn[r] : 0.0) - Bn * W[q] * cn[q];
      }
      K[r * cols + nu] = flux ? (cn[r] - u_n) : 1.0;
      b[r] = known + seed_T;
    }
    lsq_solve(Q9, cols, K, b, x);
    for (int a = 0; a < nu; ++a) gk[unk[a]] = x[a];
    if (flux) kappa = x[nu];
    if (mult) mult[2] = x[nu];
  }

  /* flow system: cols = nu + 2 */
  int cols = nu + 2;
  double K[Q9 * 8], b[Q9], x[8];
  double t[2] = {-n[1], n[0]};
  double s = 0.0;
  if (m & TAG_J_INLET) s += seed_dp;
  if (m & TAG_J_OUTLET) s -= seed_dp;
  for (int r = 0; r < Q9; ++r) {
    double known = 0.0;
    for (int q = 0; q < Q9; ++q) {
      double cc = CX[q] * CX[r] + CY[q] * CY[r];
      double coef = (q == r ? cn[r] : 0.0) - 2.0 * A * W[q] * cn[q] * cc;
      if (cn[q] <= 0) known += coef * fk[q];
    }
    for (int a = 0; a < nu; ++a) {
      int q = unk[a];
      double cc = CX[q] * CX[r] + CY[q] * CY[r];
      K[r * cols + a] = (q == r ? cn[r] : 0.0) - 2.0 * A * W[q] * cn[q] * cc;
    }
    if (FLOW(m) == FLOW_VELOCITY) {
      K[r * cols + nu] = CX[r];
      K[r * cols + nu + 1] = CY[r];
    } else {
      K[r * cols + nu] = 1.0;
      K[r * cols + nu + 1] = CX[r] * t[0] + CY[r] * t[1];
    }
    b[r] = known + s - (flux ? kappa * Tn * cn[r] : 0.0);
  }
  lsq_solve(Q9, cols, K, b, x);
  for (int a = 0; a < nu; ++a) fk[unk[a]] = x[a];
  if (mult) {
    mult[0] = x[nu];
    mult[1] = x[nu + 1];
  }
}

/* ------------------------------------------------------------------ */
/* ALKS step                                                           */
/* ------------------------------------------------------------------ */
/* One ALKS step, adjoint level n+1 -> n (eq:albef, eq:albef_ex, eq:albeg,
 * eq:albeg_ex and the weighted moments eq:afp..eq:agq, equivalently the
 * update eq:ap..eq:aq).
 *
 *   f~*_i(x) = f~_i^eq(x + c_i, n+1),   g~*_i(x) = g~_i^eq(x + c_i, n+1)
 *   f~_i = f~*_i - 3 alpha c_i.u~ + 3 T c_i.q~ - dJ_O/df_i
 *   g~_i = g~*_i - dJ_O/dg_i
 * with u~, q~ and T at level n. The equilibria use (u, T) at level n+1
 * (u_src, T_src); the coupling uses T at level n (T_dst). The Brinkman term
 * is implicit in u~ like the forward one: taking sum_i w_i c_i of the f~
 * equation gives u~ (1 + alpha) = sum_i w_i c_i (f~*_i + 3 T c_i.q~ -
 * dJ_O/df_i).
 *
 * Volume seeds (heat objective, J_O = seed_heat * u_x T on probe nodes, with
 * u_x = sum c_ix f_i and T = sum g_i): dJ_O/df_i = seed_heat T c_ix,
 * dJ_O/dg_i = seed_heat u_x, evaluated at level n. Heat-exchange objective
 * J_O = -seed_src sum beta (1 - T): dJ_O/dg_i = seed_src beta. Heat-sink
 * objective (a boundary objective, seed_bt = dJ/dT at the heated ring nodes).
 * Reading: the heated node's temperature is the flux closure of the
 * populations that arrive there, T (1 + u.n) = S0 + 2 S+ + qbar, so the
 * objective's derivative with respect to the arriving g_i is
 * seed_bt w_i^cl / (1 + u.n) with w^cl = 1 for c_i.n = 0, 2 for c_i.n > 0
 * and 0 for c_i.n < 0; it is subtracted from the node's completed adjoint
 * populations like the volume seed -dJ_O/dg_i of eq:albeg_ex. Taken
 * literally as a uniform seed dJ/dg_i = seed_bt in the rows of
 * eq:agboundaryq, the gradient of the paper's natural-convection check
 * (Sec. 2.6) is uncorrelated with central differences along the design
 * domain's centre line (correlation 0.5, median ratio 0.05 after 10000
 * steps), where the paper reports fair agreement; with this reading it
 * agrees (correlation 0.97, median ratio 1.02).
 *
 * Heat source (beta non-NULL): eq:albeg_ex adds dx dQ/dg_i T~ = -beta T~ to
 * g~_i at the same level, so T~ is implicit like u~:
 * T~ (1 + beta) = sum_i w_i (g~*_i + 3 dG/dg_i . u~ - dJ_O/dg_i); q~ is
 * unchanged (sum_i w_i c_i = 0). In exact mode the division moves to Theta
 * (orc_adjoint_equilibrium).
 *
 * Ring nodes: the pulled values are known for c_i.n <= 0, the rest come
 * from boundary_fill; alpha = 0 there and the coupling and seeds act on the
 * completed set as in the interior (reading). Corners copy the adjoint
 * moments of their neighbour along y (reading). */
void orc_alks_step(const orc_problem *P, const double *alpha, const double *B,
                   const double *beta, const double *ux_src, const double *uy_src,
                   const double *T_src, const double *ux_dst,
                   const double *uy_dst, const double *T_dst,
                   const double *const *adj_in, double *const *adj_out,
                   double seed_dp, double seed_heat, double seed_src,
                   double seed_bt, double *work) {
  const int nx = P->nx, ny = P->ny, N = nx * ny;
  const double A = coef_A(P);
  const int th = P->thermal;
  double *Vx = work, *Vy = work + N, *Th = work + 2 * N;
  orc_adjoint_equilibrium(P, B, ux_src, uy_src, adj_in, Vx, Vy, th ? Th : NULL,
                          P->adj_exact ? alpha : NULL, beta);

#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j) {
    for (int i = 0; i < nx; ++i) {
      int k = idx(P, i, j);
      /* in a periodic box every node is interior; only the tags count */
      uint8_t m = P->periodic ? (P->mask[k] & ~15) : P->mask[k];
      if (FLOW(m) == FLOW_CORNER) continue;
      int nrm[2] = {0, 0};
      int bnd = on_ring(P, i, j);
      if (bnd) ring_normal(P, i, j, &nrm[0], &nrm[1]);

      double fs[Q9], gs[Q9];
      for (int q = 0; q < Q9; ++q) {
        int cn = CX[q] * nrm[0] + CY[q] * nrm[1];
        fs[q] = 0.0;
        gs[q] = 0.0;
        if (bnd && cn > 0) continue; /* unknown, filled below */
        int kz = nbr(P, i, j, CX[q], CY[q]);
        fs[q] = adj_in[A_R][kz] + CX[q] * Vx[kz] + CY[q] * Vy[kz];
        if (th) gs[q] = Th[kz];
      }
      double Tn = th ? T_dst[k] : 0.0;
      if (bnd) {
        boundary_fill(P, m, nrm, A, B[k], Tn, ux_dst[k], uy_dst[k], seed_dp, 0.0, fs, gs,
                      NULL);
        if (th && (m & TAG_PROBE) && seed_bt != 0.0) {
          double un = ux_dst[k] * nrm[0] + uy_dst[k] * nrm[1];
          for (int q = 0; q < Q9; ++q) {
            int cn = CX[q] * nrm[0] + CY[q] * nrm[1];
            double wcl = cn == 0 ? 1.0 : (cn > 0 ? 2.0 : 0.0);
            gs[q] -= seed_bt * wcl / (1.0 + un);
          }
        }
      }

      /* volume seeds at level n */
      double dJdf[Q9] = {0}, dJdg = 0.0;
      if (m & TAG_PROBE) {
        for (int q = 0; q < Q9; ++q) dJdf[q] = seed_heat * Tn * CX[q];
        dJdg = seed_heat * ux_dst[k];
      }
      if (beta) dJdg += seed_src * beta[k];
      /* g~ and its moments */
      double Tt = 0, qx = 0, qy = 0;
      if (th) {
        for (int q = 0; q < Q9; ++q) {
          double g = gs[q] - dJdg;
          Tt += W[q] * g;
          qx += W[q] * CX[q] * g;
          qy += W[q] * CY[q] * g;
        }
        /* exact mode: the temperature of a prescribed-temperature node does
         * not depend on the populations that arrive there, so their adjoint
         * vanishes (T~ = q~ = 0) in place of the least-squares completion
         * of eq:agboundaryT; without it a conductivity contrast next to
         * such a wall makes the adjoint grow without bound */
        if (bnd && P->adj_exact && THERM(m) == THERM_DIRICHLET) Tt = qx = qy = 0.0;
      }
      /* f~ (without the implicit Brinkman part) and its moments */
      double r = 0, Ux = 0, Uy = 0, sxx = 0, sxy = 0, syy = 0;
      for (int q = 0; q < Q9; ++q) {
        double f = fs[q] + 3.0 * Tn * (CX[q] * qx + CY[q] * qy) - dJdf[q];
        r += W[q] * f;
        Ux += W[q] * CX[q] * f;
        Uy += W[q] * CY[q] * f;
        sxx += W[q] * CX[q] * CX[q] * f;
        sxy += W[q] * CX[q] * CY[q] * f;
        syy += W[q] * CY[q] * CY[q] * f;
      }
      /* paper: u~ = U~ / (1 + alpha) here; exact: the division is applied to
       * V at this node before the next pull */
      double inv = P->adj_exact ? 1.0 : 1.0 / (1.0 + alpha[k]);
      /* paper: the Boussinesq coupling 3 dG/dg_i . u~ of eq:albeg_ex adds
       * 3 g beta . u~ to T~ at interior nodes (sum_i w_i = 1) */
      if (th && !bnd && !P->adj_exact)
        Tt += 3.0 * (P->gbeta[0] * Ux + P->gbeta[1] * Uy) * inv;
      /* paper: the implicit heat source, T~ = (...) / (1 + beta) */
      if (th && beta && !P->adj_exact) Tt /= 1.0 + beta[k];
      adj_out[A_R][k] = r;
      adj_out[A_UX][k] = Ux * inv;
      adj_out[A_UY][k] = Uy * inv;
      adj_out[A_SXX][k] = sxx;
      adj_out[A_SXY][k] = sxy;
      adj_out[A_SYY][k] = syy;
      adj_out[A_T][k] = Tt;
      adj_out[A_QX][k] = qx;
      adj_out[A_QY][k] = qy;
    }
  }
  if (P->periodic) return;
  for (int k = 0; k < N; ++k) {
    if (FLOW(P->mask[k]) != FLOW_CORNER) continue;
    int i = k % nx, j = k / nx;
    int kn = idx(P, i, j == 0 ? 1 : ny - 2);
    for (int f = 0; f < A_NF; ++f) adj_out[f][k] = adj_out[f][kn];
  }
}

/* ------------------------------------------------------------------ */
/* sensitivity                                                         */
/* ------------------------------------------------------------------ */
/* Adds weight * (3 alpha'(gamma) u.u~ - B'(gamma) grad T . q~) at every
 * design (interior) node: the integrand of <J', dgamma> in Sec. 2.5 with
 * G = Q = 0 and dJ_O/dgamma = 0, in lattice units. In exact mode the
 * Brinkman part is alpha' u.V / (1 + alpha), with V the undivided
 * coefficient of eq:afeq: the derivative of u = U* / (1 + alpha) in alpha
 * paired with the adjoint of u. */
void orc_sens_add(const orc_problem *P, const double *alpha, const double *dalpha,
                  const double *dB, const double *ux, const double *uy, const double *T,
                  const double *const *adj, double weight, double *sens) {
  const int nx = P->nx, ny = P->ny;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j) {
    for (int i = 0; i < nx; ++i) {
      int k = idx(P, i, j);
      if (on_ring(P, i, j)) continue;
      double v;
      if (P->adj_exact) {
        double V[2];
        adj_V(P, i, j, ux, uy, adj, V);
        v = dalpha[k] * (ux[k] * V[0] + uy[k] * V[1]) / (1.0 + alpha[k]);
      } else {
        v = 3.0 * dalpha[k] * (ux[k] * adj[A_UX][k] + uy[k] * adj[A_UY][k]);
      }
      if (P->thermal && T) {
        double dTx = ddx(P, T, i, j, 0), dTy = ddx(P, T, i, j, 1);
        v -= dB[k] * (dTx * adj[A_QX][k] + dTy * adj[A_QY][k]);
      }
      sens[k] += weight * v;
    }
  }
}

/* Adds the heat-source part of the sensitivity integrand of Sec. 2.5 at
 * every design node: dJ_O/dgamma - dx dQ/dgamma T~ with Q = beta (1 - T)
 * and the heat-exchange objective J_O = -w_J sum beta (1 - T), i.e.
 *   beta'(gamma) (T - 1) (w_J + T~)
 * (w_J = 0 for other objectives). In exact mode T~ is replaced by the
 * propagated Theta of the node (divided by 1 + beta), the adjoint of T*
 * paired with dT/dbeta = (1 - T) / (1 + beta). */
void orc_source_sens_add(const orc_problem *P, const double *alpha, const double *B,
                         const double *beta, const double *dbeta, const double *ux,
                         const double *uy, const double *T, const double *const *adj,
                         double wJ, double *sens) {
  const int nx = P->nx, ny = P->ny, N = nx * ny;
  double *Th = NULL, *Vx = NULL, *Vy = NULL;
  if (P->adj_exact) {
    Th = malloc(3 * (size_t)N * sizeof(double));
    Vx = Th + N;
    Vy = Th + 2 * N;
    orc_adjoint_equilibrium(P, B, ux, uy, adj, Vx, Vy, Th, alpha, beta);
  }
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      int k = idx(P, i, j);
      if (on_ring(P, i, j)) continue;
      double a = P->adj_exact ? Th[k] : adj[A_T][k];
      sens[k] += dbeta[k] * (T[k] - 1.0) * (wJ + a);
    }
  free(Th);
}

/* Exported so that tests can reach the boundary fill directly. mult
 * receives the flow multipliers (mu~_x, mu~_y) or (lambda~, mu~_s) and the
 * thermal multiplier (eta~ or kappa~). */
void orc_boundary_fill(const orc_problem *P, uint8_t m, int nx_, int ny_,
                       double Bn, double Tn, double unx, double uny,
                       double seed_dp, double *fk, double *gk, double *mult,
                       double seed_T) {
  int n[2] = {nx_, ny_};
  boundary_fill(P, m, n, coef_A(P), Bn, Tn, unx, uny, seed_dp, seed_T, fk, gk, mult);
}

/* OpenMP thread count of the oracle's loops (timing on 1 core and on all) */
void orc_set_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
