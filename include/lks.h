/*
 * lks.h -- C ABI of the MI355X (gfx950) library for the Lattice Kinetic
 * Scheme (LKS) forward step and its adjoint (ALKS) sweep, which produce the
 * flow and thermal fields and the design sensitivity dJ/dgamma for
 * Brinkman-penalised topology optimisation (Tanabe, Yaji and Ushijima,
 * "Adjoint lattice kinetic scheme for topology optimization in fluid
 * problems", arXiv 2411.03090).
 *
 * The calls follow the optimisation procedure of Sec. 2.7: Step 2 (state by
 * LKS) is lks_forward, Step 3 (objective) is lks_objective, Steps 4-5
 * (adjoint fields by ALKS and the sensitivity) are alks_backward.
 *
 * Conventions shared by every call
 *   - Lattice units dx = dt = 1, relaxation times tau_f = tau_g = 1 (Sec. 2.4).
 *   - D2Q9 lattice; fields are node arrays of nx*ny values, x fastest:
 *     node (i, j) is element j*nx + i. The outer ring of nodes is the
 *     boundary; its class comes from the node-class byte below, its outward
 *     normal from its position.
 *   - D3Q19 extension (the same equations with the indices running over
 *     x, y, z, Sec. 2.1): fields of nx*ny*nz values, node (i, j, l) is
 *     element (l*ny + j)*nx + i. A node at an end of a non-periodic axis is
 *     a boundary node: a face node when one coordinate is at an end (outward
 *     normal along that axis), an edge or corner node when two or three are.
 *   - Device pointers are plain HIP device addresses (for example the
 *     data_ptr() of a torch tensor on the same device); host pointers are
 *     ordinary memory. The library never frees caller memory.
 *   - Every call returns an lks_status and never throws. On an error the
 *     context keeps its previous state and lks_last_error() holds a message.
 *   - Calls are asynchronous on the HIP stream given to lks_create, except
 *     lks_objective and the sizing/report calls. A context is not thread
 *     safe; distinct contexts are independent.
 */
#ifndef LKS_H_
#define LKS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lks_ctx lks_ctx;

typedef enum {
  LKS_OK = 0,
  LKS_E_INVALID = 1,     /* bad argument or parameter outside the scheme's range */
  LKS_E_NOMEM = 2,       /* workspace or memory budget too small */
  LKS_E_HIP = 3,         /* a HIP runtime call failed */
  LKS_E_STATE = 4,       /* call out of order (e.g. backward before forward) */
  LKS_E_DIVERGED = 5,    /* non-finite state detected */
  LKS_E_UNSUPPORTED = 6  /* valid request this build does not implement */
} lks_status;

/* lattice and precision */
enum { LKS_D2Q9 = 0, LKS_D3Q19 = 1 };
/* FP64: state and arithmetic in double.
 * FP32DEV: state in float with the density stored as rho - 1; objective and
 * sensitivity accumulated in double.
 * MIXED (steady D2Q9 problems): the forward sweep and the objective in
 * double, the adjoint sweep in float (FP32DEV) from the final forward state
 * rounded to float once; the sensitivity accumulated in double. The forward
 * fields and J are those of FP64; the gradient carries the FP32 adjoint's
 * error. */
enum { LKS_FP64 = 0, LKS_FP32DEV = 1, LKS_MIXED = 2 };
/* objectives: static pressure drop (eq:objective_pipebend); time-averaged
 * enthalpy flux u_x T through the probe nodes; heat-exchange amount
 * J = -sum beta_gamma (1 - T) over all nodes (eq:objective_heatexchanger;
 * needs the heat source, beta_max > 0); heat-sink objective: the mean
 * temperature over the heated boundary (eq:objective_heatsink; D2Q9), whose
 * adjoint seed follows the heated node's flux closure: seed w / (1 + u.n)
 * per arriving population, w = 1 along the wall and 2 moving outwards */
enum { LKS_OBJ_PRESSURE_DROP = 0, LKS_OBJ_HEAT = 1, LKS_OBJ_HEAT_EXCHANGE = 2,
       LKS_OBJ_HEAT_SINK = 3 };
enum { LKS_STEADY = 0, LKS_UNSTEADY = 1 };
enum { LKS_ADJ_PAPER = 0, LKS_ADJ_EXACT = 1 };
/* checkpointing of unsteady sweeps (see lks_set_checkpointing) */
enum { LKS_CKPT_AUTO = 0, LKS_CKPT_TWO_LEVEL = 1, LKS_CKPT_BINOMIAL = 2 };

/* Node-class byte (one per node):
 *   bits 0-1 flow class: interior (design) node, prescribed velocity
 *            (inlet or wall), prescribed pressure (outlet), corner (D2Q9) /
 *            edge or corner (D3Q19): u = 0, density, temperature and adjoint
 *            moments copied from the neighbour one step inwards along y
 *            (and z);
 *   bits 2-3 thermal class: none, prescribed temperature, prescribed heat
 *            flux -q.n = q_bar with q = sum_i c_i g_i - u T (Sec. 2.4), q_bar
 *            read from T_bar at the node (0: adiabatic);
 *   bit 4/5  member of the inlet/outlet set of the pressure drop
 *            (eq:objective_pipebend);
 *   bit 6    member of the probe set of the heat-transfer objective, or
 *            of the heated boundary of the heat-sink objective (ring nodes
 *            of the heat-flux class);
 *   bit 7    D3Q19 only: interior node that is not a design node (its
 *            sensitivity is zero), e.g. a solid held at a prescribed
 *            temperature (interior node with thermal class "prescribed
 *            temperature": T = T_bar, adjoint T~ = q~ = 0).
 * Sec. 2.4 names the boundary conditions (velocity at inlets and walls,
 * pressure and tangential velocity at outlets, temperature or heat flux). */
#define LKS_FLOW_INTERIOR 0
#define LKS_FLOW_VELOCITY 1
#define LKS_FLOW_PRESSURE 2
#define LKS_FLOW_CORNER 3
#define LKS_THERM_DIRICHLET (1 << 2)
#define LKS_THERM_FLUX (2 << 2)
#define LKS_TAG_J_INLET (1 << 4)
#define LKS_TAG_J_OUTLET (1 << 5)
#define LKS_TAG_PROBE (1 << 6)
#define LKS_TAG_SOLID (1 << 7)

/* Fields for lks_read_field / lks_write_field. Forward state: density
 * deviation rho - 1, velocity, temperature, at the current level. Adjoint
 * state: the coefficients of the adjoint equilibria at the current adjoint
 * level, f~_i^eq = rho~ + c_i . V (eq:afeq) and g~_i^eq = Theta (eq:ageq). */
enum {
  LKS_FIELD_DRHO = 0,
  LKS_FIELD_UX = 1,
  LKS_FIELD_UY = 2,
  LKS_FIELD_T = 3,
  LKS_FIELD_ADJ_RHO = 4,
  LKS_FIELD_ADJ_VX = 5,
  LKS_FIELD_ADJ_VY = 6,
  LKS_FIELD_ADJ_THETA = 7,
  LKS_FIELD_UZ = 8,     /* D3Q19 */
  LKS_FIELD_ADJ_VZ = 9  /* D3Q19 */
};

typedef struct {
  int nx, ny, nz;  /* nodes per axis; nz = 1 for D2Q9 */
  int lattice;     /* LKS_D2Q9 or LKS_D3Q19 */
  int precision;   /* LKS_FP64, LKS_FP32DEV or LKS_MIXED */
  int periodic;    /* D2Q9: 1 = periodic box, every node interior.
                      D3Q19: mask of periodic axes (bit 0 x, 1 y, 2 z) */
} lks_grid;

typedef struct {
  double nu;          /* kinematic viscosity; A = (9/2)(1/6 - nu), eq:A */
  double Pr;          /* Prandtl number; fluid diffusivity K_f = nu / Pr */
  double alpha_max;   /* alpha-bar of eq:brinkman */
  double q_alpha;     /* q_alpha of eq:brinkman */
  double Ks_over_Kf;  /* K_s / K_f of eq:conductivity */
  double q_K;         /* q_K of eq:conductivity */
  int thermal;        /* 1: solve the temperature field too */
  double gbeta[3];    /* g beta of the Boussinesq force G = g beta (T - T_ref)
                         (eq:boussinesqforce), lattice units; all zero: no
                         force. Non-zero needs a thermal D2Q9 problem (D3Q19:
                         LKS_E_UNSUPPORTED); the third component is unused */
  double T_ref;       /* reference temperature of the Boussinesq force */
  double beta_max;    /* beta-bar of the heat source Q = beta_gamma (1 - T)
                         (eq:heatsource, eq:betagamma) that heats the solid;
                         0: no source. Positive needs a thermal D2Q9 problem
                         (D3Q19: LKS_E_UNSUPPORTED) */
  double q_beta;      /* q_beta of eq:betagamma (> 0 when beta_max > 0) */
} lks_phys;

typedef struct {
  const uint8_t *node_class; /* host, one class per node (copied) */
  const double *u_bar;       /* host, 2 (D3Q19: 3) blocks of one value per
                                node: x block, y block (, z block); the
                                velocity prescribed at velocity nodes (copied) */
  const double *T_bar;       /* host, one value per node: temperature at
                                prescribed-T nodes, heat flux into the
                                domain at heat-flux nodes, ignored elsewhere
                                (copied); may be NULL if not thermal */
  const double *u_factor;    /* host, n_factor: u_bar is scaled by
                                u_factor[min(n, n_factor-1)] at level n;
                                NULL means 1 (copied) */
  int n_factor;
  double rho_out;            /* prescribed outlet density (p = rho/3) */
  int objective;             /* LKS_OBJ_* */
  int mode;                  /* LKS_STEADY or LKS_UNSTEADY */
  int n_steps;               /* unsteady: steps N of the horizon (levels
                                0..N); steady: ignored */
} lks_bc;

/* Create a context. Validates the problem (Sec. 2.4 ranges: 0 < nu < 1/6,
 * 0 <= K_s, K_f <= 1/6, alpha_max >= 0, q > 0, |u_bar| <= 0.3, node classes
 * consistent with the ring) and plans the memory: for unsteady problems the
 * trajectory (u, T) is kept either whole or as checkpoints every K levels
 * with K chosen as the largest interval whose storage fits
 * mem_budget_bytes (0 = no limit). Makes no HIP call. hip_stream is a
 * hipStream_t (NULL = the null stream). On success *out owns host memory
 * only; bind a device workspace before computing. */
lks_status lks_create(const lks_grid *grid, const lks_phys *phys, const lks_bc *bc,
                      size_t mem_budget_bytes, void *hip_stream, lks_ctx **out);

/* Bytes of device workspace the context needs (state, adjoint, design
 * coefficients, boundary data, checkpoints and replay segment). */
lks_status lks_workspace_size(const lks_ctx *ctx, size_t *bytes);

/* Bind caller-owned device memory of at least lks_workspace_size bytes,
 * 256-byte aligned. Uploads the boundary data. The memory must outlive the
 * context's use. */
lks_status lks_bind_workspace(lks_ctx *ctx, void *dev_ptr, size_t bytes);

/* Size of the library's static per-device workspace array (64 MiB). */
#define LKS_STATIC_WORKSPACE_BYTES (64u * 1024u * 1024u)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): bind the context
 * to the library's static workspace array on the current device instead of
 * caller memory, then use the context as after lks_bind_workspace. The array
 * (LKS_STATIC_WORKSPACE_BYTES, 256-byte aligned) is part of the library's
 * code object: each device holds its own copy from the first load of the
 * library until the process ends; this call allocates no device memory
 * (no hipMalloc, hipFree or allocating library routine), it uploads the
 * boundary data and clears the state like lks_bind_workspace.
 * One array per device is shared by every context: binding a context makes
 * the context bound to it before on that device unusable (its calls return
 * LKS_E_STATE until it is bound again), and calls of two contexts that
 * overlap in time on one device race. The array keeps the last context's
 * contents; everything a sweep needs cleared is cleared by the sweep.
 * Errors: LKS_E_NOMEM when lks_workspace_size exceeds
 * LKS_STATIC_WORKSPACE_BYTES (nothing is bound), LKS_E_HIP when the array's
 * device address cannot be obtained. */
lks_status lks_bind_static_workspace(lks_ctx *ctx);

/* Step 2: reset to the level-0 state (rho = 1, u = 0, T = 0 inside, the
 * prescribed values on the boundary) and run `steps` LKS steps
 * (eq:rho, eq:u, eq:T with eq:feq2, eq:geq2 and the implicit Brinkman term
 * of eq:lbef_ex) for the design gamma_dev (device, nx*ny doubles in [0,1]).
 * Unsteady contexts require steps == n_steps and store the trajectory. */
lks_status lks_forward(lks_ctx *ctx, const double *gamma_dev, int steps);

/* Continue the current forward state by `steps` steps without reset and
 * without trajectory storage (steady contexts; parity and convergence runs). */
lks_status lks_advance(lks_ctx *ctx, const double *gamma_dev, int steps);

/* Step 3: the objective of the last forward run, in double. Steady: on the
 * final state. Unsteady: averaged over levels 1..N. Synchronises the stream. */
lks_status lks_objective(lks_ctx *ctx, double *J_host);

/* Steps 4-5: ALKS adjoint sweep (eq:ap..eq:aq with eq:afeq, eq:ageq and the
 * least-squares adjoint boundary treatment of Sec. 2.5 / Appendix A) and
 * the sensitivity (Sec. 2.5) written to dJdgamma_dev (device, nx*ny doubles,
 * overwritten; zero on boundary nodes). Linear in J_seed. The boundary seed
 * of the pressure-drop objective (dJ/df_i in eq:afboundaryu and
 * eq:afboundaryp) is J_seed per unit boundary pressure, +J_seed on inlet
 * nodes and -J_seed on outlet nodes, the reading under which the gradient of
 * the paper's non-thermal check (Sec. 2.6) agrees with central differences.
 * Steady: adj_steps ALKS steps with the state frozen at the last forward
 * level and the seed applied every step, then the sensitivity once.
 * Unsteady: adj_steps is ignored; the sweep runs from the terminal condition
 * f~ = g~ = 0 down to level 0, replaying checkpoint segments, and sums the
 * sensitivity over levels. Returns LKS_E_STATE before a forward run. */
lks_status alks_backward(lks_ctx *ctx, double J_seed, int adj_steps, double *dJdgamma_dev);

/* Synchronises the stream and reports LKS_E_DIVERGED when the last forward
 * state or the sensitivity of the last adjoint sweep holds a non-finite value
 * (with a large conductivity contrast next to a prescribed-temperature wall
 * the paper's least-squares completion of eq:agboundaryT feeds a growing
 * thermal adjoint mode; the exact adjoint mode, which zeroes the thermal
 * adjoint there, stays bounded), LKS_E_STATE before an adjoint sweep, LKS_OK
 * otherwise. */
lks_status lks_gradient_status(lks_ctx *ctx);

/* Continue the steady adjoint by `steps` ALKS steps from its current state
 * (no reset), with the state frozen at the current forward level; writes the
 * sensitivity of the final level when dJdgamma_dev is not NULL. */
lks_status alks_advance(lks_ctx *ctx, double J_seed, int steps, double *dJdgamma_dev);

/* Copy field `which` (LKS_FIELD_*) of the current level to dev_out
 * (device, nx*ny doubles). Asynchronous. */
lks_status lks_read_field(lks_ctx *ctx, int which, double *dev_out);

/* Overwrite field `which` of the current level from dev_in (device, nx*ny
 * doubles), e.g. to start a step from a prescribed state. Asynchronous. */
lks_status lks_write_field(lks_ctx *ctx, int which, const double *dev_in);

/* Tile autotuner: times `steps` forward and `steps` adjoint steps of the
 * design gamma_dev for each launch shape the kernels provide (tiles of
 * 64 x 4, 64 x 8 and, where supported, 64 x 16 nodes; one or, where
 * supported, two steps per launch)
 * on this context's stream, keeps the fastest and reports its tile height in
 * *tile_rows (lks_launch_shape gives the whole shape). Synchronises; the forward and adjoint states are discarded
 * (run lks_forward afterwards). D2Q9 only (LKS_E_UNSUPPORTED for D3Q19,
 * whose node-parallel kernels have no tile shape). */
lks_status lks_autotune(lks_ctx *ctx, const double *gamma_dev, int steps, int *tile_rows);

/* Set the tile height (4 or 8 rows of 64 nodes, or 16 for FP32 non-thermal
 * problems) explicitly; results do not depend on it. Discards the forward and
 * adjoint states. D2Q9 only. Two steps per launch apply to heights 4 and 8;
 * with 16 every launch runs one step. */
lks_status lks_set_tile_rows(lks_ctx *ctx, int tile_rows);

/* Time steps per kernel launch, forward (lks_advance, lks_forward, and the
 * checkpoint replays of an unsteady alks_backward) and adjoint (steady
 * alks_backward, alks_advance; an unsteady adjoint sweep runs one step per
 * launch): 1, or 2 for FP32 D2Q9 problems and for the forward sweep of FP64
 * non-thermal D2Q9 problems (LKS_E_UNSUPPORTED otherwise; a MIXED context
 * applies forward_steps to its FP64 forward and adjoint_steps to its FP32
 * adjoint). With 2, each launch loads its tile with a 4-node halo and runs
 * two steps, the first on the tile and a 2-node halo kept in LDS; an unsteady
 * sweep stores from there what a checkpoint or replay slot keeps of the level
 * between. The states are bitwise those of one step per launch; an unsteady
 * objective sums the same terms per tile and level, in another order within
 * a tile. */
lks_status lks_set_steps_per_launch(lks_ctx *ctx, int forward_steps, int adjoint_steps);

/* Adjoint formulation used by alks_backward and alks_advance.
 * LKS_ADJ_PAPER (default): the ALKS of Sec. 2.5, where the implicit Brinkman
 * division acts on u~ at the node where the adjoint moments are formed
 * (eq:albef_ex) and the sensitivity pairs 3 alpha'(gamma) u.u~.
 * LKS_ADJ_EXACT: the transpose of the discrete LKS step u = U* / (1 + alpha).
 * u~ stays undivided, the coefficient V of eq:afeq is divided by 1 + alpha at
 * its own node before it propagates, the Brinkman part of the sensitivity is
 * alpha' u.V / (1 + alpha) with the undivided V, and an unsteady sweep sums
 * the sensitivity over levels 1..N only (level 0 is the initial state). On
 * periodic grids with uniform B this gives the exact discrete gradient; ring
 * and face nodes keep the paper's least-squares completion, except that the
 * thermal adjoint of a prescribed-temperature node is zero (its temperature
 * does not depend on the populations that arrive there). Changing the
 * mode discards the adjoint state. Batches take lks_batch_set_adjoint_mode.
 * Errors: LKS_E_INVALID for another value. */
lks_status lks_set_adjoint_mode(lks_ctx *ctx, int mode);

/* D3Q19 contexts: run each ALKS step (eq:afeq, eq:ageq, eq:afp - eq:agq and
 * the sensitivity) as one z-marching kernel over the interior planes, which
 * keeps the adjoint moments of a plane in LDS and registers (fused = 1, the
 * default), or as a pull pass, a face pass and an update pass that store the
 * moments of every node between them (fused = 0). Both give the same bits;
 * boundary nodes take the face pass's moments either way. Errors:
 * LKS_E_UNSUPPORTED for D2Q9 contexts, LKS_E_INVALID for another value. */
lks_status lks_set_fused_adjoint(lks_ctx *ctx, int fused);

/* The launch shape in use: tile height (0 for D3Q19) and steps per launch of
 * the forward and adjoint sweeps. */
lks_status lks_launch_shape(const lks_ctx *ctx, int *tile_rows, int *forward_steps,
                            int *adjoint_steps);

/* Memory plan: bytes of checkpoint + replay storage, bytes of the rest of
 * the workspace, and the checkpoint interval K (N when the whole trajectory
 * is stored; 0 for steady problems). */
lks_status lks_memory_report(const lks_ctx *ctx, size_t *ckpt_bytes, size_t *state_bytes,
                             int *K);

/* Checkpointing of an unsteady context (the paper keeps every level of the
 * trajectory, Sec. 3.2 and 3.4; this library trades memory for recomputed
 * forward steps). Call before lks_bind_workspace; it re-plans the workspace
 * (query lks_workspace_size again).
 *   LKS_CKPT_TWO_LEVEL: checkpoints of the whole state every K levels and one
 *     replay segment of K-1 levels, K the interval that fits the budget
 *     with the fewest replayed steps (K = N+1, the whole trajectory, when it
 *     fits); the adjoint recomputes at most one forward sweep.
 *   LKS_CKPT_BINOMIAL: `slots` snapshots of the whole state besides level 0
 *     (0: as many as the budget holds) placed by Griewank's binomial
 *     reversal schedule, which recomputes the fewest forward steps possible
 *     for that many snapshots; for budgets where two-level does not fit.
 *   LKS_CKPT_AUTO (the default at lks_create): two-level when it fits the
 *     budget, binomial otherwise.
 * Results are bitwise the same under every scheme. Errors: LKS_E_STATE after
 * binding, LKS_E_UNSUPPORTED for steady contexts, LKS_E_INVALID for an
 * unknown scheme or slots < 0 (slots > 0 needs LKS_CKPT_BINOMIAL),
 * LKS_E_NOMEM when the plan exceeds the budget of lks_create (the previous
 * plan is kept). */
lks_status lks_set_checkpointing(lks_ctx *ctx, int scheme, int slots);

/* The plan of an unsteady context: scheme (LKS_CKPT_TWO_LEVEL or
 * LKS_CKPT_BINOMIAL), count (the interval K, or the number of snapshots
 * including level 0) and the LKS steps one adjoint sweep recomputes. Steady
 * contexts report zeros. */
lks_status lks_checkpoint_info(const lks_ctx *ctx, int *scheme, int *count,
                               long long *replay_steps);

/* ---- batches (Sec. 2.7 Steps 2-5 for many independent designs) ----------
 * A batch holds n D2Q9 problems of possibly different sizes and parameters
 * (same precision and mode, all thermal or all non-thermal, no heat source):
 *   steady batches: the pressure-drop objective; one call runs n_fwd LKS
 *     steps, the objective, n_adj ALKS steps and the sensitivity of every
 *     design;
 *   unsteady batches: the pressure-drop or enthalpy-flux objective averaged
 *     over levels 1..N, with one horizon N (lks_bc.n_steps) for all designs;
 *     one call runs the N LKS steps, the objectives and the whole checkpointed
 *     adjoint sweep (two-level checkpointing with one interval K for every
 *     design, chosen by lks_batch_set_memory_budget), the sensitivity summed
 *     over levels as alks_backward does for one design.
 * Each step of all designs is one kernel launch, and the whole sequence is
 * captured once as a HIP graph and replayed (use_graph = 1) or launched
 * eagerly (use_graph = 0). Each design's results are bitwise those of its own
 * context at the same tile height. */
typedef struct lks_batch lks_batch;

/* Validates every design as lks_create does. Makes no HIP call. grids/phys/bcs
 * are arrays of n descriptors. An unsteady batch starts with every level kept
 * (no budget). Errors: LKS_E_UNSUPPORTED for other lattices, objectives,
 * MIXED precision or a heat source; LKS_E_INVALID when the designs differ in
 * precision, physics kind, mode or horizon. */
lks_status lks_batch_create(int n, const lks_grid *grids, const lks_phys *phys,
                            const lks_bc *bcs, void *hip_stream, lks_batch **out);
/* Device memory budget of the whole batch (workspace bytes; 0 = no limit),
 * before binding. Unsteady batches take the checkpoint interval that replays
 * the fewest forward steps within it (as lks_create plans one design).
 * Errors: LKS_E_STATE after binding, LKS_E_NOMEM when no plan fits (the
 * previous plan is kept). Makes no HIP call. */
lks_status lks_batch_set_memory_budget(lks_batch *b, size_t bytes);
/* Adjoint mode of every design (as lks_set_adjoint_mode); default paper. */
lks_status lks_batch_set_adjoint_mode(lks_batch *b, int mode);
/* The plan: checkpoint interval K and LKS steps one sweep replays (0 and 0
 * for steady batches), and the workspace bytes. Any pointer may be NULL. */
lks_status lks_batch_checkpoint_info(const lks_batch *b, int *K, long long *replay_steps,
                                     size_t *workspace_bytes);
lks_status lks_batch_workspace_size(const lks_batch *b, size_t *bytes);
/* Bind caller-owned device memory (256-byte aligned); creates the batch's
 * internal capture stream and events. */
lks_status lks_batch_bind_workspace(lks_batch *b, void *dev_ptr, size_t bytes);
/* gamma_dev[d], dJdgamma_dev[d]: device pointers of design d (nx*ny doubles);
 * J_host: n doubles. Synchronises the stream. Linear in J_seed. Unsteady
 * batches need n_fwd == n_steps; n_adj = 0 runs the forward sweep and the
 * objectives only (dJdgamma_dev untouched), any other n_adj the whole
 * adjoint sweep. */
lks_status lks_batch_run(lks_batch *b, const double *const *gamma_dev, int n_fwd, int n_adj,
                         double J_seed, double *const *dJdgamma_dev, double *J_host,
                         int use_graph);
/* Tile autotuner of a steady batch: runs the batch eagerly for `steps`
 * forward and adjoint steps per tile height and keeps the fastest.
 * scratch_dev[d] receives a throw-away sensitivity. Synchronises. Unsteady
 * batches: LKS_E_UNSUPPORTED. */
lks_status lks_batch_autotune(lks_batch *b, const double *const *gamma_dev, int steps,
                              double *const *scratch_dev, int *tile_rows);
/* Tile height of a batch's step launches (as lks_set_tile_rows; 4 or 8 for
 * unsteady batches). */
lks_status lks_batch_set_tile_rows(lks_batch *b, int tile_rows);
/* Field `which` of design d at its final forward / adjoint level (unsteady
 * batches: adjoint fields only, those of level 0; LKS_E_UNSUPPORTED for
 * forward fields, whose last levels the replays overwrite). */
lks_status lks_batch_read_field(lks_batch *b, int design, int which, double *dev_out);
const char *lks_batch_last_error(const lks_batch *b);
void lks_batch_destroy(lks_batch *b);

const char *lks_strerror(lks_status s);
const char *lks_last_error(const lks_ctx *ctx);
void lks_destroy(lks_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* LKS_H_ */
