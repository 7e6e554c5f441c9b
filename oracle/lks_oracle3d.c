/*
 * Plain FP64 CPU oracle of the three-dimensional (D3Q19) extension of the
 * Lattice Kinetic Scheme and its adjoint.
 *
 * TEST INFRASTRUCTURE ONLY, like lks_oracle.c: the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it; the product
 * path never does. It shares no code with the GPU library (and none with
 * the two-dimensional oracle either: this file stands alone).
 *
 * The paper is two-dimensional; its equations are written with indices
 * alpha, beta that run over x, y (and x, y, z in three dimensions, Sec. 2.1).
 * This file takes every equation of Sec. 2.3-2.5 unchanged with the D3Q19
 * velocity set, whose weights satisfy the same isotropy conditions as D2Q9
 * (sum w c_a c_b = delta_ab / 3 and the fourth-order condition), so eq:A and
 * eq:B hold unchanged:
 *   c0 = 0                                          w = 1/3
 *   c1..c6   = +x -x +y -y +z -z                    w = 1/18
 *   c7..c18  = (+-1,+-1,0), (+-1,0,+-1), (0,+-1,+-1) w = 1/36
 * Projecting D3Q19 along z (summing the weights of directions with equal
 * (c_x, c_y)) gives D2Q9 with its weights, so a z-invariant run reproduces the
 * two-dimensional scheme.
 *
 * Geometry: nodes (i, j, l), k = (l ny + j) nx + i. Axis x, y, z is periodic
 * when the corresponding bit of `periodic` is set. A node is a boundary node
 * when it sits at an end of a non-periodic axis. Its node-class byte says how:
 *   flow class 1 (velocity) or 2 (pressure): a face node, one coordinate at
 *     an end; the outward normal follows from the position;
 *   flow class 3 (copy): an edge or corner node, two or three coordinates at
 *     an end. Reading (the analogue of the two-dimensional corner rule): u = 0,
 *     and rho, T and the adjoint moments are copied from the node reached by
 *     stepping inwards along y and z, (i, j', l'), at the new level.
 * Interior nodes may carry the temperature class "Dirichlet" (a solid block
 * at fixed temperature): the forward T is set to Tbar after the pull, and the
 * adjoint temperature moments (T~, q~) are zero there (reading). Interior
 * nodes tagged SOLID are not design nodes: their sensitivity is zero.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q19 19

static const int C3[Q19][3] = {
    {0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
    {-1, 0, 1}, {0, 1, 1},   {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static double w3(int q) {
  if (q == 0) return 1.0 / 3.0;
  if (q <= 6) return 1.0 / 18.0;
  return 1.0 / 36.0;
}

#define FLOW(m) ((m) & 3)
#define FLOW_VELOCITY 1
#define FLOW_PRESSURE 2
#define FLOW_COPY 3
#define THERM(m) (((m) >> 2) & 3)
#define THERM_DIRICHLET 1
#define THERM_FLUX 2
#define TAG_J_INLET 16
#define TAG_J_OUTLET 32
#define TAG_PROBE 64
#define TAG_SOLID 128

typedef struct {
  int nx, ny, nz;
  int periodic;              /* bit 0: x, bit 1: y, bit 2: z */
  int thermal;
  double nu;                 /* eq:A */
  double Kf, Ks, q_K;        /* eq:conductivity */
  double alpha_max, q_alpha; /* eq:brinkman */
  double rho_out;
  const uint8_t *mask;       /* nx*ny*nz node classes */
  const double *ubar;        /* 3 N prescribed velocity (x, y, z blocks) */
  const double *Tbar;        /* N prescribed temperature */
  int adj_exact;             /* 1: exact discrete adjoint of the Brinkman step */
} orc3_problem;

static inline int n_of(const orc3_problem *P, int a) {
  return a == 0 ? P->nx : a == 1 ? P->ny : P->nz;
}
static inline int per(const orc3_problem *P, int a) { return (P->periodic >> a) & 1; }
static inline long idx3(const orc3_problem *P, int i, int j, int l) {
  return ((long)l * P->ny + j) * P->nx + i;
}
static inline void coords(const orc3_problem *P, long k, int x[3]) {
  x[0] = (int)(k % P->nx);
  x[1] = (int)((k / P->nx) % P->ny);
  x[2] = (int)(k / ((long)P->nx * P->ny));
}

/* neighbour of x shifted by d, or -1 outside a non-periodic axis */
static long nbr3(const orc3_problem *P, const int x[3], const int d[3]) {
  int y[3];
  for (int a = 0; a < 3; ++a) {
    int n = n_of(P, a);
    y[a] = x[a] + d[a];
    if (per(P, a)) y[a] = (y[a] % n + n) % n;
    else if (y[a] < 0 || y[a] >= n) return -1;
  }
  return idx3(P, y[0], y[1], y[2]);
}

/* number of coordinates at an end of a non-periodic axis; the outward
 * normal when there is exactly one */
static int ends(const orc3_problem *P, const int x[3], int nrm[3]) {
  int c = 0;
  for (int a = 0; a < 3; ++a) {
    nrm[a] = 0;
    if (per(P, a)) continue;
    if (x[a] == 0) { nrm[a] = -1; ++c; }
    else if (x[a] == n_of(P, a) - 1) { nrm[a] = 1; ++c; }
  }
  return c;
}

/* the node an edge or corner node copies from: inwards along y and z */
static long copy_source(const orc3_problem *P, const int x[3]) {
  int y[3] = {x[0], x[1], x[2]};
  for (int a = 1; a < 3; ++a) {
    if (per(P, a)) continue;
    if (y[a] == 0) y[a] = 1;
    else if (y[a] == n_of(P, a) - 1) y[a] = n_of(P, a) - 2;
  }
  return idx3(P, y[0], y[1], y[2]);
}

/* F5 stencil along axis a: central inside (or periodic), second-order
 * one-sided at the two ends of a non-periodic axis */
static double dd3(const orc3_problem *P, const double *f, const int x[3], int a) {
  int n = n_of(P, a), p = x[a];
  int e[3] = {0, 0, 0};
  if (per(P, a) || (p > 0 && p < n - 1)) {
    e[a] = 1;
    double fp = f[nbr3(P, x, e)];
    e[a] = -1;
    return 0.5 * (fp - f[nbr3(P, x, e)]);
  }
  int s = p == 0 ? 1 : -1;
  e[a] = s;
  double f1 = f[nbr3(P, x, e)];
  e[a] = 2 * s;
  double f2 = f[nbr3(P, x, e)];
  return 0.5 * s * (-3.0 * f[idx3(P, x[0], x[1], x[2])] + 4.0 * f1 - f2);
}

static double coef_A3(const orc3_problem *P) { return 4.5 * (1.0 / 6.0 - P->nu); }

static int is_boundary(const orc3_problem *P, long k) {
  int x[3], n[3];
  coords(P, k, x);
  return ends(P, x, n) > 0;
}

/* eq:brinkman, eq:conductivity, eq:B; boundary nodes are non-design fluid
 * nodes (alpha = 0, B = B(Kf)); SOLID nodes keep their coefficients but have
 * zero derivatives. */
void orc3_coefficients(const orc3_problem *P, const double *gamma, double *alpha,
                       double *dalpha, double *B, double *dB) {
  long N = (long)P->nx * P->ny * P->nz;
  for (long k = 0; k < N; ++k) {
    if (is_boundary(P, k)) {
      alpha[k] = 0.0;
      dalpha[k] = 0.0;
      B[k] = 3.0 * (1.0 / 6.0 - P->Kf);
      dB[k] = 0.0;
      continue;
    }
    double g = gamma[k], qa = P->q_alpha, qk = P->q_K;
    alpha[k] = P->alpha_max * qa * (1.0 - g) / (qa + g);
    dalpha[k] = -P->alpha_max * qa * (1.0 + qa) / ((qa + g) * (qa + g));
    double K = P->Kf + (P->Ks - P->Kf) * qk * (1.0 - g) / (qk + g);
    double dK = -(P->Ks - P->Kf) * qk * (1.0 + qk) / ((qk + g) * (qk + g));
    B[k] = 3.0 * (1.0 / 6.0 - K);
    dB[k] = -3.0 * dK;
    if (P->mask[k] & TAG_SOLID) {
      dalpha[k] = 0.0;
      dB[k] = 0.0;
    }
  }
}

/* eq:feq2 with drho in place of rho (the constant w_i adds 1 to the density
 * and nothing to the momentum) */
static double feq3(int q, double drho, const double u[3], const double G[3][3], double A) {
  double cu = 0, uu = 0, strain = 0;
  for (int a = 0; a < 3; ++a) {
    cu += C3[q][a] * u[a];
    uu += u[a] * u[a];
    for (int b = 0; b < 3; ++b) strain += (G[a][b] + G[b][a]) * C3[q][a] * C3[q][b];
  }
  return w3(q) * (drho + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu + A * strain);
}

/* eq:geq2, linear reading w_i [T (1 + 3 c.u) + B c.grad T] */
static double geq3(int q, double T, const double u[3], double B, const double dT[3]) {
  double cu = 0, cd = 0;
  for (int a = 0; a < 3; ++a) {
    cu += C3[q][a] * u[a];
    cd += C3[q][a] * dT[a];
  }
  return w3(q) * (T * (1.0 + 3.0 * cu) + B * cd);
}

/* level-0 state: rho = 1, u = 0 (ubar * ufac0 on velocity faces), T = 0
 * (Tbar on temperature nodes), copy nodes copying T */
void orc3_init_state(const orc3_problem *P, double ufac0, double *drho, double *u,
                     double *T) {
  long N = (long)P->nx * P->ny * P->nz;
  for (long k = 0; k < N; ++k) {
    drho[k] = 0.0;
    for (int a = 0; a < 3; ++a) u[a * N + k] = 0.0;
    if (T) T[k] = 0.0;
    uint8_t m = P->mask[k];
    int x[3], n[3];
    coords(P, k, x);
    if (ends(P, x, n) == 1 && FLOW(m) == FLOW_VELOCITY)
      for (int a = 0; a < 3; ++a) u[a * N + k] = P->ubar[a * N + k] * ufac0;
    if (T && THERM(m) == THERM_DIRICHLET) T[k] = P->Tbar[k];
  }
  if (!T) return;
  for (long k = 0; k < N; ++k) {
    int x[3], n[3];
    coords(P, k, x);
    if (ends(P, x, n) >= 2) T[k] = T[copy_source(P, x)];
  }
}

/* One LKS step n -> n+1 (the same equations as the two-dimensional oracle:
 * eq:rho, eq:u, eq:T; implicit Brinkman u = U* / (1 + alpha); face closures
 * by moment balance over the pulled populations with c_i.n >= 0). State
 * arrays: drho (N), u (3 N: x, y, z blocks), T (N). */
void orc3_lks_step(const orc3_problem *P, const double *alpha, const double *B,
                   double ufac, const double *drho, const double *u, const double *T,
                   double *drho_o, double *u_o, double *T_o) {
  const long N = (long)P->nx * P->ny * P->nz;
  const double A = coef_A3(P);
  const int th = P->thermal;
#pragma omp parallel for schedule(static)
  for (long k = 0; k < N; ++k) {
    int x[3], nrm[3];
    coords(P, k, x);
    int ne = ends(P, x, nrm);
    if (ne >= 2) continue;
    uint8_t m = P->mask[k];
    double rho_s = 0, U[3] = {0, 0, 0}, T_s = 0;
    double S0 = 0, Sp = 0, S0g = 0, Spg = 0;
    for (int q = 0; q < Q19; ++q) {
      int cn = C3[q][0] * nrm[0] + C3[q][1] * nrm[1] + C3[q][2] * nrm[2];
      if (ne && cn < 0) continue;
      int d[3] = {-C3[q][0], -C3[q][1], -C3[q][2]};
      long kz = nbr3(P, x, d);
      int z[3];
      coords(P, kz, z);
      double uz[3] = {u[kz], u[N + kz], u[2 * N + kz]};
      double G[3][3];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) G[a][b] = dd3(P, u + a * N, z, b);
      double f = feq3(q, drho[kz], uz, G, A);
      double g = 0.0;
      if (th) {
        double dT[3] = {dd3(P, T, z, 0), dd3(P, T, z, 1), dd3(P, T, z, 2)};
        g = geq3(q, T[kz], uz, B[kz], dT);
      }
      rho_s += f;
      for (int a = 0; a < 3; ++a) U[a] += C3[q][a] * f;
      T_s += g;
      if (cn == 0) { S0 += f; S0g += g; }
      if (cn > 0) { Sp += f; Spg += g; }
    }
    if (!ne) {
      drho_o[k] = rho_s;
      for (int a = 0; a < 3; ++a) u_o[a * N + k] = U[a] / (1.0 + alpha[k]);
      if (th) T_o[k] = THERM(m) == THERM_DIRICHLET ? P->Tbar[k] : T_s;
      continue;
    }
    double un = 0.0;
    if (FLOW(m) == FLOW_VELOCITY) {
      for (int a = 0; a < 3; ++a) {
        u_o[a * N + k] = P->ubar[a * N + k] * ufac;
        un += u_o[a * N + k] * nrm[a];
      }
      drho_o[k] = S0 + 2.0 * Sp - un;
    } else {
      double dro = P->rho_out - 1.0;
      drho_o[k] = dro;
      un = S0 + 2.0 * Sp - dro;
      for (int a = 0; a < 3; ++a) u_o[a * N + k] = un * nrm[a];
    }
    if (th) {
      if (THERM(m) == THERM_DIRICHLET) T_o[k] = P->Tbar[k];
      /* heat-flux face: -q.n = qbar (Tbar holds qbar there; 0: adiabatic) */
      else T_o[k] = (S0g + 2.0 * Spg + P->Tbar[k]) / (1.0 + un);
    }
  }
  for (long k = 0; k < N; ++k) {
    int x[3], nrm[3];
    coords(P, k, x);
    if (ends(P, x, nrm) < 2) continue;
    long ks = copy_source(P, x);
    drho_o[k] = drho_o[ks];
    for (int a = 0; a < 3; ++a) u_o[a * N + k] = 0.0;
    if (th) T_o[k] = T_o[ks];
  }
}

double orc3_pressure_drop(const orc3_problem *P, const double *drho) {
  long N = (long)P->nx * P->ny * P->nz;
  double s = 0.0;
  for (long k = 0; k < N; ++k) {
    if (P->mask[k] & TAG_J_INLET) s += (1.0 + drho[k]) / 3.0;
    if (P->mask[k] & TAG_J_OUTLET) s -= (1.0 + drho[k]) / 3.0;
  }
  return s;
}

double orc3_probe_heat(const orc3_problem *P, const double *u, const double *T) {
  long N = (long)P->nx * P->ny * P->nz;
  double s = 0.0;
  for (long k = 0; k < N; ++k)
    if (P->mask[k] & TAG_PROBE) s += u[k] * T[k];
  return s;
}

/* Adjoint state: 14 arrays of N
 *   0 rho~  1-3 u~  4 s~xx 5 s~xy 6 s~xz 7 s~yy 8 s~yz 9 s~zz  10 T~  11-13 q~ */
enum { R3 = 0, U3 = 1, S3 = 4, T3 = 10, Q3 = 11, NF3 = 14 };
static const int SIDX[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};

/* eq:afeq, eq:ageq with three components:
 *   V_a = 3 u~_a + 9 s~_ab u_b - 3 rho~ u_a - 2A d_b s~_ab
 *   Theta = T~ + 3 q~.u - B div q~ - grad B . q~ */
/* V_a at node k (x its coordinates) from the adjoint moments and the state u */
static void adj_V3(const orc3_problem *P, long k, const int x[3], const double *u,
                   const double *const *adj, double V[3]) {
  const long N = (long)P->nx * P->ny * P->nz;
  const double A = coef_A3(P);
  double uk[3] = {u[k], u[N + k], u[2 * N + k]};
  for (int a = 0; a < 3; ++a) {
    double su = 0, ds = 0;
    for (int b = 0; b < 3; ++b) {
      const double *s = adj[S3 + SIDX[a][b]];
      su += s[k] * uk[b];
      ds += dd3(P, s, x, b);
    }
    V[a] = 3.0 * adj[U3 + a][k] + 9.0 * su - 3.0 * adj[R3][k] * uk[a] - 2.0 * A * ds;
  }
}

/* With alpha given (exact mode), V is divided by 1 + alpha at its node. In
 * exact mode (the problem's flag) the thermal term is the transpose
 * -div_h (B q~) of the forward B c.grad_h T (see the D2Q9 oracle). */
void orc3_adjoint_equilibrium(const orc3_problem *P, const double *B, const double *u,
                              const double *const *adj, double *V, double *Theta,
                              const double *alpha) {
  const long N = (long)P->nx * P->ny * P->nz;
  double *Bq = NULL;
  if (Theta && P->adj_exact) {
    Bq = malloc(3 * (size_t)N * sizeof(double));
    for (int a = 0; a < 3; ++a)
      for (long k = 0; k < N; ++k) Bq[a * N + k] = B[k] * adj[Q3 + a][k];
  }
#pragma omp parallel for schedule(static)
  for (long k = 0; k < N; ++k) {
    int x[3];
    coords(P, k, x);
    double uk[3] = {u[k], u[N + k], u[2 * N + k]};
    double Vk[3];
    adj_V3(P, k, x, u, adj, Vk);
    const double sc = alpha ? 1.0 / (1.0 + alpha[k]) : 1.0;
    for (int a = 0; a < 3; ++a) V[a * N + k] = Vk[a] * sc;
    if (Theta) {
      double qu = 0, divq = 0, gbq = 0, dbq = 0;
      for (int a = 0; a < 3; ++a) {
        qu += adj[Q3 + a][k] * uk[a];
        divq += dd3(P, adj[Q3 + a], x, a);
        gbq += dd3(P, B, x, a) * adj[Q3 + a][k];
        if (Bq) dbq += dd3(P, Bq + a * N, x, a);
      }
      Theta[k] = Bq ? adj[T3][k] + 3.0 * qu - dbq
                    : adj[T3][k] + 3.0 * qu - B[k] * divq - gbq;
    }
  }
  free(Bq);
}

/* least squares min ||K x + b|| by the normal equations (Gaussian
 * elimination with partial pivoting) */
static void lsq3(int rows, int cols, const double *K, const double *b, double *x) {
  double G[12][13];
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

/* Adjoint face fill (Sec. 2.5, Appendix A), the rows of the two-dimensional
 * reading over the 19 directions:
 *   flow:    (n.c_i) f~_i - 2A sum_j w_j (n.c_j)(c_j.c_i) f~_j
 *            + [mu~.c_i | lambda~ + mu~_1 (c_i.t1) + mu~_2 (c_i.t2)]
 *            - kappa~ T (c_i.n) + s_i
 *   thermal: (n.c_i) g~_i - B sum_j w_j (n.c_j) g~_j + [eta~ | kappa~ (c_i - u).n]
 * with t1, t2 the two coordinate axes normal to n. Unknowns: the five
 * directions with c_i.n > 0 and the multipliers; least squares over all 19
 * rows. fk, gk hold the known values (c_i.n <= 0) and are completed in
 * place; mult receives the flow multipliers (3) and the thermal one. */
static void fill3(const orc3_problem *P, uint8_t m, const int n[3], double A, double Bn,
                  double Tn, const double u[3], double seed_dp, double *fk, double *gk,
                  double *mult) {
  double cn[Q19];
  int unk[Q19], nu = 0;
  for (int q = 0; q < Q19; ++q) {
    cn[q] = C3[q][0] * n[0] + C3[q][1] * n[1] + C3[q][2] * n[2];
    if (cn[q] > 0) unk[nu++] = q;
  }
  double kappa = 0.0;
  int flux = P->thermal && THERM(m) == THERM_FLUX;
  if (P->thermal) {
    int cols = nu + 1;
    double K[Q19 * 12], b[Q19], x[12];
    double un = u[0] * n[0] + u[1] * n[1] + u[2] * n[2];
    for (int r = 0; r < Q19; ++r) {
      double known = 0.0;
      for (int q = 0; q < Q19; ++q) {
        double coef = (q == r ? cn[r] : 0.0) - Bn * w3(q) * cn[q];
        if (cn[q] <= 0) known += coef * gk[q];
      }
      for (int a = 0; a < nu; ++a) {
        int q = unk[a];
        K[r * cols + a] = (q == r ? cn[r] : 0.0) - Bn * w3(q) * cn[q];
      }
      K[r * cols + nu] = flux ? (cn[r] - un) : 1.0;
      b[r] = known;
    }
    lsq3(Q19, cols, K, b, x);
    for (int a = 0; a < nu; ++a) gk[unk[a]] = x[a];
    if (flux) kappa = x[nu];
    if (mult) mult[3] = x[nu];
  }
  int ax = n[0] ? 0 : n[1] ? 1 : 2;
  int t1 = (ax + 1) % 3, t2 = (ax + 2) % 3;
  int cols = nu + 3;
  double K[Q19 * 12], b[Q19], x[12];
  double s = 0.0;
  /* the boundary seed per unit pressure, as in the D2Q9 fill */
  if (m & TAG_J_INLET) s += seed_dp;
  if (m & TAG_J_OUTLET) s -= seed_dp;
  for (int r = 0; r < Q19; ++r) {
    double known = 0.0;
    for (int q = 0; q < Q19; ++q) {
      double cc = C3[q][0] * C3[r][0] + C3[q][1] * C3[r][1] + C3[q][2] * C3[r][2];
      double coef = (q == r ? cn[r] : 0.0) - 2.0 * A * w3(q) * cn[q] * cc;
      if (cn[q] <= 0) known += coef * fk[q];
    }
    for (int a = 0; a < nu; ++a) {
      int q = unk[a];
      double cc = C3[q][0] * C3[r][0] + C3[q][1] * C3[r][1] + C3[q][2] * C3[r][2];
      K[r * cols + a] = (q == r ? cn[r] : 0.0) - 2.0 * A * w3(q) * cn[q] * cc;
    }
    if (FLOW(m) == FLOW_VELOCITY) {
      for (int a = 0; a < 3; ++a) K[r * cols + nu + a] = C3[r][a];
    } else {
      K[r * cols + nu] = 1.0;
      K[r * cols + nu + 1] = C3[r][t1];
      K[r * cols + nu + 2] = C3[r][t2];
    }
    b[r] = known + s - (flux ? kappa * Tn * cn[r] : 0.0);
  }
  lsq3(Q19, cols, K, b, x);
  for (int a = 0; a < nu; ++a) fk[unk[a]] = x[a];
  if (mult)
    for (int a = 0; a < 3; ++a) mult[a] = x[nu + a];
}

/* One ALKS step, adjoint level n+1 -> n (eq:albef_ex, eq:albeg_ex, the
 * weighted moments eq:afp..eq:agq with 19 directions), as in the
 * two-dimensional oracle: the equilibria use (u, T) at level n+1 (u_src,
 * T_src), the coupling, Brinkman and seeds the level n (u_dst, T_dst).
 * work: 4 N doubles. */
void orc3_alks_step(const orc3_problem *P, const double *alpha, const double *B,
                    const double *u_src, const double *T_src, const double *u_dst,
                    const double *T_dst, const double *const *adj_in,
                    double *const *adj_out, double seed_dp, double seed_heat,
                    double *work) {
  (void)T_src;
  const long N = (long)P->nx * P->ny * P->nz;
  const double A = coef_A3(P);
  const int th = P->thermal;
  double *V = work, *Th = work + 3 * N;
  orc3_adjoint_equilibrium(P, B, u_src, adj_in, V, th ? Th : NULL, P->adj_exact ? alpha : NULL);
#pragma omp parallel for schedule(static)
  for (long k = 0; k < N; ++k) {
    int x[3], nrm[3];
    coords(P, k, x);
    int ne = ends(P, x, nrm);
    if (ne >= 2) continue;
    uint8_t m = P->mask[k];
    double fs[Q19], gs[Q19];
    for (int q = 0; q < Q19; ++q) {
      int cn = C3[q][0] * nrm[0] + C3[q][1] * nrm[1] + C3[q][2] * nrm[2];
      fs[q] = 0.0;
      gs[q] = 0.0;
      if (ne && cn > 0) continue;
      long kz = nbr3(P, x, C3[q]);
      fs[q] = adj_in[R3][kz] + C3[q][0] * V[kz] + C3[q][1] * V[N + kz] + C3[q][2] * V[2 * N + kz];
      if (th) gs[q] = Th[kz];
    }
    double Tn = th ? T_dst[k] : 0.0;
    double ud[3] = {u_dst[k], u_dst[N + k], u_dst[2 * N + k]};
    if (ne) fill3(P, m, nrm, A, B[k], Tn, ud, seed_dp, fs, gs, NULL);
    double dJdf[Q19] = {0}, dJdg = 0.0;
    if (m & TAG_PROBE) {
      for (int q = 0; q < Q19; ++q) dJdf[q] = seed_heat * Tn * C3[q][0];
      dJdg = seed_heat * ud[0];
    }
    double Tt = 0, qv[3] = {0, 0, 0};
    if (th) {
      for (int q = 0; q < Q19; ++q) {
        double g = gs[q] - dJdg;
        Tt += w3(q) * g;
        for (int a = 0; a < 3; ++a) qv[a] += w3(q) * C3[q][a] * g;
      }
      /* the temperature of a prescribed-temperature node does not depend
       * on the populations that arrive there, so their adjoint vanishes:
       * inside the domain in both modes, and on faces in the exact mode
       * (the paper's least-squares completion of eq:agboundaryT there
       * otherwise) */
      if (THERM(m) == THERM_DIRICHLET && (!ne || P->adj_exact)) {
        Tt = 0.0;
        qv[0] = qv[1] = qv[2] = 0.0;
      }
    }
    double r = 0, U[3] = {0, 0, 0}, s[6] = {0, 0, 0, 0, 0, 0};
    for (int q = 0; q < Q19; ++q) {
      double cq = C3[q][0] * qv[0] + C3[q][1] * qv[1] + C3[q][2] * qv[2];
      double f = fs[q] + 3.0 * Tn * cq - dJdf[q];
      double wf = w3(q) * f;
      r += wf;
      for (int a = 0; a < 3; ++a) {
        U[a] += C3[q][a] * wf;
        for (int b = a; b < 3; ++b) s[SIDX[a][b]] += C3[q][a] * C3[q][b] * wf;
      }
    }
    double inv = P->adj_exact ? 1.0 : 1.0 / (1.0 + alpha[k]);
    adj_out[R3][k] = r;
    for (int a = 0; a < 3; ++a) adj_out[U3 + a][k] = U[a] * inv;
    for (int c = 0; c < 6; ++c) adj_out[S3 + c][k] = s[c];
    adj_out[T3][k] = Tt;
    for (int a = 0; a < 3; ++a) adj_out[Q3 + a][k] = qv[a];
  }
  for (long k = 0; k < N; ++k) {
    int x[3], nrm[3];
    coords(P, k, x);
    if (ends(P, x, nrm) < 2) continue;
    long ks = copy_source(P, x);
    for (int f = 0; f < NF3; ++f) adj_out[f][k] = adj_out[f][ks];
  }
}

/* weight * (3 alpha' u.u~ - B' grad T . q~) at every design node */
void orc3_sens_add(const orc3_problem *P, const double *alpha, const double *dalpha,
                   const double *dB, const double *u, const double *T,
                   const double *const *adj, double weight, double *sens) {
  const long N = (long)P->nx * P->ny * P->nz;
#pragma omp parallel for schedule(static)
  for (long k = 0; k < N; ++k) {
    int x[3], nrm[3];
    coords(P, k, x);
    if (ends(P, x, nrm) > 0 || (P->mask[k] & TAG_SOLID)) continue;
    double v = 0.0;
    if (P->adj_exact) {
      /* alpha' u.V / (1 + alpha) with the undivided V */
      double Vk[3];
      adj_V3(P, k, x, u, adj, Vk);
      for (int a = 0; a < 3; ++a) v += u[a * N + k] * Vk[a];
      v *= dalpha[k] / (1.0 + alpha[k]);
    } else {
      for (int a = 0; a < 3; ++a) v += u[a * N + k] * adj[U3 + a][k];
      v *= 3.0 * dalpha[k];
    }
    if (P->thermal && T)
      for (int a = 0; a < 3; ++a) v -= dB[k] * dd3(P, T, x, a) * adj[Q3 + a][k];
    sens[k] += weight * v;
  }
}

/* the face fill of one node, exported for tests */
void orc3_boundary_fill(const orc3_problem *P, uint8_t m, int n0, int n1, int n2, double Bn,
                        double Tn, double u0, double u1, double u2, double seed_dp,
                        double *fk, double *gk, double *mult) {
  int n[3] = {n0, n1, n2};
  double u[3] = {u0, u1, u2};
  fill3(P, m, n, coef_A3(P), Bn, Tn, u, seed_dp, fk, gk, mult);
}
