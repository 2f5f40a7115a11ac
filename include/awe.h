/*
 * awe.h - acoustic wave-equation forward operator, its adjoint and the adjoint-state
 * gradient on AMD Instinct MI355X (gfx950).  C ABI; no C++ or framework types.
 *
 * Operations (paper: section "Wave-equation-based inversion", equation eq-fwi and the
 * two Julia listings that follow it - the JUDI gradient-descent loop and the rrule
 * whose pullback returns (J^T dy, F^T dy)):
 *
 *   forward   d  = F(m) q,      F(m) = P_r A(m)^{-1} P_s^T   (m = squared slowness)
 *   adjoint   v  = F(m)^T dd                                 (gradient w.r.t. the source)
 *   gradient  g  = J(m, q)^T dd                              (gradient w.r.t. m; with
 *                  dd = F(m) q - d_obs it is the gradient of 1/2 ||F(m) q - d_obs||^2)
 *   born      dd = J(m, q) dm                                (linearised data)
 *
 * Discretisation (the paper gives none; these are the library's definitions):
 *   - computational grid = physical grid + nbl cells on both ends of every axis;
 *     arrays are row-major [nz][nx] (2D) or [nz][ny][nx] (3D), x fastest; fields are
 *     zero outside the computational grid;
 *   - L_h = 8th-order central Laplacian (weights -205/72, 8/5, -1/5, 8/315, -1/560 per
 *     axis, divided by h^2);
 *   - damping eta = sum over axes of 3 ln(1/R) / (2 nbl h vref) (d/nbl)^2 with d the
 *     number of cells past the inner edge of the border (0 inside);
 *   - row k = 1..nt-1 of A u = s, with u^0 = u^{-1} = 0:
 *       (m/dt^2 + eta/(2dt)) u^k - (2m/dt^2 + L_h) u^{k-1} + (m/dt^2 - eta/(2dt)) u^{k-2}
 *         = s^{k-1};
 *   - P_s^T q: s^n = R(x_s)^T q^n / h^ndim; P_r u: d^n = R(x_r) u^n for n = 0..nt-1,
 *     R = bilinear (2D) / trilinear (3D) interpolation weights;
 *   - adjoint: A^T w = P_r^T dd solved backward from w^nt = w^{nt+1} = 0;
 *     v^n = R(x_s) w^{n+1} / h^ndim for n = 0..nt-2 and v^{nt-1} = 0;
 *   - gradient: g = -(1/dt^2) sum_j u^j (w^j - 2 w^{j+1} + w^{j+2}) summed over the shots
 *     of each model window in ascending shot order (FP64 accumulation).
 *
 * Units: h in m, time in ms, m in ms^2/m^2 (= s^2/km^2), velocities in km/s, positions
 * in m in the physical coordinates of the shot's model window (x = i h for physical
 * column i).
 *
 * Ownership and streams: every array argument except the problem description is a
 * device pointer owned by the caller.  The library allocates device memory only in
 * awe_plan_create (its geometry tables, freed by awe_plan_destroy); calls on the
 * compute path never allocate.  All compute calls enqueue on the given hipStream_t
 * (NULL = default stream) and return without synchronising; inputs must stay valid
 * until the stream reaches the work.  Calls on one workspace must not overlap.
 *
 * Errors: every function returns an awe_status; nothing throws across the ABI.  On
 * error no work has been enqueued and awe_last_error() returns a thread-local message.
 */
#ifndef AWE_H
#define AWE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AWE_VERSION 1

typedef enum {
  AWE_OK = 0,
  AWE_ERR_INVALID_ARG = 1,  /* null pointer, bad size, bad enum value */
  AWE_ERR_UNSUPPORTED = 2,  /* valid request that the library does not implement */
  AWE_ERR_CFL = 3,          /* vmax dt / h above the leapfrog stability limit */
  AWE_ERR_GEOMETRY = 4,     /* source or receiver outside the computational grid */
  AWE_ERR_WORKSPACE = 5,    /* workspace null or smaller than awe_plan_workspace_size */
  AWE_ERR_STATE = 6,        /* awe_backward without a preceding awe_forward(keep=1) */
  AWE_ERR_HIP = 7,          /* a HIP runtime call failed */
  AWE_ERR_NONFINITE = 8,    /* screening on (awe_plan_set_checks): an input or output holds a
                               value that is not finite */
  AWE_ERR_INTERNAL = 9      /* launch checks on (awe_plan_set_checks): a launch would touch bytes
                               outside its workspace sub-buffer or tables (a library defect) */
} awe_status;

/* One shot: a model window, its time axis and its acquisition. */
typedef struct {
  int32_t nx, ny, nz;   /* computational grid of the window (physical + 2 nbl); ny = 1 in 2D */
  int32_t nt;           /* time samples t_n = n dt, n = 0..nt-1 (nt >= 2) */
  int64_t m_offset;     /* element offset of the window in m, dm and g */
  int64_t q_offset;     /* element offset of the shot's nt samples in q and v */
  int64_t d_offset;     /* element offset of the shot's traces [nt][nrec] in d and dd */
  int64_t rec_offset;   /* row of the shot's first receiver in awe_problem.rec_pos */
  int32_t nrec;         /* receivers of this shot (>= 0) */
  int32_t reserved0;
  double src[3];        /* source position (x, y, z) in m; y ignored in 2D */
} awe_shot;

typedef struct {
  int32_t ndim;          /* 2 or 3 */
  int32_t nbl;           /* damping border width in cells (>= 0) */
  double h;              /* grid spacing, m */
  double dt;             /* time step, ms */
  double vmax;           /* bound on the velocity 1/sqrt(m) of every model passed (km/s) */
  double damp_vref;      /* reference velocity of the damping profile (km/s) */
  double damp_R;         /* target reflection coefficient, 0 < R <= 1 (1 = no damping) */
  int32_t nshot;
  int32_t reserved0;
  const awe_shot* shots; /* host array [nshot]; copied by awe_plan_create */
  const double* rec_pos; /* host array [rows][3] of (x, y, z); copied by awe_plan_create */
} awe_problem;

typedef enum {
  AWE_STORE_NONE = 0,       /* forward only: no wavefield kept (forward, adjoint, born) */
  AWE_STORE_FULL = 1,       /* every u^n kept in the workspace */
  AWE_STORE_CHECKPOINT = 2, /* nslots restart pairs (u^n, u^{n-1}) per shot, binomial
                               recomputation schedule */
  AWE_STORE_AUTO = 3,       /* FULL if its workspace fits the memory budget, else CHECKPOINT
                               with the most restart slots per shot that fit (at most nslots
                               when nslots > 0, at most the number of time steps); the plan
                               reports the choice (awe_plan_get_storage) */
  AWE_STORE_PROBED = 4      /* no wavefield kept: nslots = r probes of the time axis (1..64),
                               2 r FP64 fields per shot; gradients by awe_gradient_probed */
} awe_store_mode;

typedef enum {
  AWE_PREC_FP32 = 0,
  AWE_PREC_BF16 = 1,  /* stored value = RNE(u / s), s = max |u| of that field (FP32) */
  AWE_PREC_FP16 = 2   /* as BF16, in IEEE half precision (subnormals kept) */
} awe_store_prec;

typedef struct {
  int32_t mode;        /* awe_store_mode */
  int32_t nslots;      /* CHECKPOINT: restart slots per shot (>= 1); AUTO: at most this many
                          (0: no limit); ignored otherwise */
  int32_t prec;        /* awe_store_prec of the stored wavefield */
  int32_t budget_mib;  /* AUTO: workspace budget in MiB; 0 = 90 % of the current device's free
                          memory at plan creation (hipMemGetInfo).  Ignored otherwise. */
} awe_storage;

typedef struct awe_plan awe_plan;

/* Validate the problem, build geometry tables (device copies allocated here), choose
 * tile shapes and lay out the workspace.  Uses the current HIP device.
 * Shots may have different nt: their time axes are aligned at the last sample.
 * Errors: INVALID_ARG, CFL, GEOMETRY, UNSUPPORTED (CHECKPOINT storage in 3D, also when AUTO
 * would need it), WORKSPACE (AUTO: not even one restart slot per shot fits the budget), HIP. */
awe_status awe_plan_create(const awe_problem* prob, const awe_storage* store, awe_plan** plan);

/* The storage awe_plan_create would put in effect for (prob, store) and the workspace bytes
 * it needs, without creating a plan.  Runs on the host only (no device call) unless store is
 * AUTO with budget_mib = 0, which reads the device's free memory.  Same errors as
 * awe_plan_create, GEOMETRY and HIP table uploads aside. */
awe_status awe_storage_select(const awe_problem* prob, const awe_storage* store, awe_storage* chosen,
                              size_t* ws_bytes);

/* The storage in effect for the plan: the one requested, or for AUTO the FULL or
 * CHECKPOINT storage it resolved to (mode, nslots, prec; budget_mib 0). */
awe_status awe_plan_get_storage(const awe_plan* plan, awe_storage* out);

/* Optional screening of caller arrays (flags, default 0 = off):
 *   AWE_CHECK_INPUTS:  before any compute work, m, q, dd and dm (those the call reads) are
 *     checked for values that are not finite (error NONFINITE), and m for values below
 *     1/vmax^2 by more than one part in 10^6, i.e. velocities above the plan's vmax, for which
 *     the leapfrog may be unstable (error CFL).  No compute work is enqueued on error.
 *   AWE_CHECK_OUTPUTS: after the call's work, d, g, v and dd (those it writes) are checked for
 *     values that are not finite (error NONFINITE; the outputs are then invalid).
 *   AWE_CHECK_LAUNCHES: before every launch the host checks what it computed for it against
 *     the plan's layout: each workspace fill and checkpoint-slot copy lies inside one
 *     sub-buffer, a step's levels lie in 1..nsteps, its tiles belong to the current shot group,
 *     restore and store slots exist, and 3D injection ranges lie inside their table.  A failed
 *     check returns INTERNAL before that launch (work already enqueued stays enqueued).  Host
 *     cost only (about a microsecond per launch and tile list); no synchronisation.
 * With INPUTS or OUTPUTS set the compute calls synchronise the stream once per screened group of
 * arrays and must not be captured into a graph.  Each screened element is read once more from
 * HBM.  Errors: INVALID_ARG, HIP (counter allocation on first use). */
enum { AWE_CHECK_INPUTS = 1, AWE_CHECK_OUTPUTS = 2, AWE_CHECK_LAUNCHES = 4 };
awe_status awe_plan_set_checks(awe_plan* plan, int32_t flags);

/* Bytes of device workspace every compute call on this plan needs (256-byte aligned
 * pointer required).  Inside the workspace every field row (nx values) is padded to a
 * multiple of 64 elements; FULL storage keeps nt such padded fields per shot, e.g.
 * nt * ceil(nx/64)*64 * ny * nz * 4 bytes in FP32.  The caller's arrays are not padded. */
awe_status awe_plan_workspace_size(const awe_plan* plan, size_t* bytes);

/* Free the plan and its device tables.  NULL is ignored. */
void awe_plan_destroy(awe_plan* plan);

/* d = F(m) q for every shot.  m: float [sum of windows] squared slowness; q: float
 * wavelets at q_offset; d: float traces [nt][nrec] at d_offset (written).
 * keep = 1 also stores the wavefield in the workspace (per the plan's storage mode)
 * for a following awe_backward on the same workspace, m and q. */
awe_status awe_forward(awe_plan* plan, const float* m, const float* q, float* d, int keep,
                       void* ws, size_t ws_bytes, void* stream);

/* Reverse sweep after awe_forward(keep = 1) on the same workspace, m and q: g = J^T dd
 * (FP64, written on every window a shot uses, other elements untouched; may be NULL) and
 * v = F^T dd (float at q_offset; may be NULL).  dd: float [nt][nrec] per shot at
 * d_offset.  q is read again when CHECKPOINT storage recomputes forward states.  FULL
 * storage keeps the forward, so backward may be repeated; CHECKPOINT consumes it.
 * Error STATE if the workspace does not hold a kept forward of this plan. */
awe_status awe_backward(awe_plan* plan, const float* m, const float* q, const float* dd, double* g,
                        float* v, void* ws, size_t ws_bytes, void* stream);

/* awe_forward(keep = 1) followed by awe_backward.  d may be NULL (traces not returned). */
awe_status awe_gradient(awe_plan* plan, const float* m, const float* q, const float* dd,
                        double* g, float* v, float* d, void* ws, size_t ws_bytes, void* stream);

/* Probed gradient: an estimate of J^T dd from r sums over the time axis instead of the stored
 * wavefield (randomized trace estimation and on-the-fly Fourier transforms, which the section
 * "Remaining challenges" cites against the memory bottleneck of the adjoint-state gradient).
 * The exact gradient is g = -(1/dt^2) sum_k w^k b^k with b^k = u^k - 2u^{k-1} + u^{k-2}
 * (k = 1..nt-1, w the adjoint field); the forward sweep accumulates B_j = sum_k C[j][k] b^k, the
 * reverse sweep A_j = sum_k C[j][k] w^k (both FP64), and g = -(1/dt^2) sum_j s_j A_j B_j: exact
 * when C^T diag(s) C = I, unbiased when its expectation is I (Rademacher rows, s_j = 1/r).
 * Plan: storage AWE_STORE_PROBED with nslots = r (2D or 3D).  C: device float [r][max_nt] row-major,
 * column k weights every shot's local level k (max_nt = the largest nt of the plan; column 0 is
 * not used).  s: host double [r], read during the call.  g: FP64 as in awe_backward; v, d (may
 * be NULL) as in awe_gradient.  One call runs the forward and the reverse sweep; no forward is
 * kept.  Workspace: the plan's (2 r FP64 fields per shot besides the field buffers).
 * Errors: INVALID_ARG, UNSUPPORTED (storage not PROBED), WORKSPACE, HIP, and the screening
 * errors of awe_plan_set_checks. */
awe_status awe_gradient_probed(awe_plan* plan, const float* m, const float* q, const float* dd,
                               const float* C, const double* s, double* g, float* v, float* d, void* ws,
                               size_t ws_bytes, void* stream);

/* v = F(m)^T dd: float [nt] per shot at q_offset. */
awe_status awe_adjoint(awe_plan* plan, const float* m, const float* dd, float* v, void* ws,
                       size_t ws_bytes, void* stream);

/* dd = J(m, q) dm (Born modelling): dm float, same layout as m; dd float traces. */
awe_status awe_born(awe_plan* plan, const float* m, const float* q, const float* dm, float* dd,
                    void* ws, size_t ws_bytes, void* stream);

/* Bytes of workspace awe_residual / awe_dot_f64 need for n elements. */
size_t awe_reduce_workspace_size(int64_t n);

/* r = d_pred - d_obs (float, may alias d_pred) and *loss = 1/2 sum r^2 accumulated in
 * FP64 (device pointer, may be NULL).  Deterministic: fixed partition and order. */
awe_status awe_residual(const float* d_pred, const float* d_obs, float* r, int64_t n,
                        double* loss, void* ws, size_t ws_bytes, void* stream);

/* awe_residual without a workspace argument, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid allocation): the
 * partial sums live in a static scratch array of the library (1024 FP64 values, 8 KiB, one copy
 * per GPU, kept until the process ends; its device address is looked up on the first call on each
 * GPU).  The scratch size does not depend on n (fixed partition), so no n >= 0 is refused.  Same
 * results as awe_residual, bit for bit.  Calls that overlap on one GPU (other streams, other
 * threads) share the scratch and race; the last call's partial sums stay in it.  Allocates
 * nothing.  Errors: INVALID_ARG (NULL input, n < 0), HIP. */
awe_status awe_residual_noalloc(const float* d_pred, const float* d_obs, float* r, int64_t n,
                                double* loss, void* stream);

/* *out = sum a_i b_i in FP64 (device pointer), deterministic. */
awe_status awe_dot_f64(const float* a, const float* b, int64_t n, double* out, void* ws,
                       size_t ws_bytes, void* stream);

/* *out = sum a_i b_i for FP64 inputs (device pointers), deterministic. */
awe_status awe_dot_f64d(const double* a, const double* b, int64_t n, double* out, void* ws,
                        size_t ws_bytes, void* stream);

/* Wavespeed parameterisation ("Putting it all together": the time-lapse operator
 * diag(F^i(v^i) q^i) is written in terms of the compressional wavespeed v, and the
 * operators of "Wave-equation-based inversion" take the squared slowness m = 1/v^2).
 * awe_slowness2: m[i] = 1/v[i]^2.  awe_velocity_gradient: the chain rule of that map,
 * gv[i] = -2 gm[i] / v[i]^3 (gm = dphi/dm, gv = dphi/dv).  float arrays of n values on the
 * device (caller-owned; gv may alias gm), computed in FP64 and rounded once.  Errors:
 * INVALID_ARG (NULL pointer, n < 0), HIP. */
awe_status awe_slowness2(const float* v, float* m, int64_t n, void* stream);
awe_status awe_velocity_gradient(const float* v, const float* gm, float* gv, int64_t n, void* stream);

/* Patchy-saturation rock physics R ("Putting it all together"): the CO2 saturation s of each
 * cell lowers its compressional wavespeed.  Per cell, with wavespeed vp (km/s), density rho
 * (kg/m^3) and porosity phi: the brine-saturated P-wave modulus P1 = rho vp^2 and shear
 * modulus mu = rho vp^2 / 3 (vs = vp / sqrt 3); Gassmann's relation in the form
 * r(K) = K / (k_min - K) gives the fully CO2-saturated bulk modulus K2 from
 * r(K2) = r(K1) - r(k_brine)/phi + r(k_co2)/phi with K1 = P1 - 4 mu / 3, and P2 = K2 + 4 mu / 3;
 * the patchy mixture's P-wave modulus is the harmonic average M = 1 / ((1 - s)/P1 + s/P2);
 * rho_new = rho + phi s (rho_co2 - rho_brine) and vp_new = sqrt(M / rho_new).
 * Constants (NULL: the paper's k_min 36.6e9, k_brine 2.735e9, k_co2 0.125e9 Pa, rho_co2 700,
 * rho_brine 1000 kg/m^3).  All arrays float, n values on the device, computed in FP64.
 * awe_patchy writes vp_new and rho_new (rho_new may be NULL); awe_patchy_vjp writes
 * g_s = g_vp dvp_new/ds + g_rho drho_new/ds (g_rho may be NULL: 0).  s = 0 returns vp and
 * rho unchanged.  n = 0 does nothing (pointers may then be NULL).  Errors: INVALID_ARG (n < 0,
 * or a required pointer NULL with n > 0), HIP. */
typedef struct {
  double k_min, k_brine, k_co2;   /* bulk moduli of the mineral, brine and CO2 (Pa) */
  double rho_co2, rho_brine;      /* fluid densities (kg/m^3) */
} awe_patchy_consts;
awe_status awe_patchy(const float* s, const float* vp, const float* rho, const float* phi, float* vp_new,
                      float* rho_new, int64_t n, const awe_patchy_consts* c, void* stream);
awe_status awe_patchy_vjp(const float* s, const float* vp, const float* rho, const float* phi,
                          const float* g_vp, const float* g_rho, float* g_s, int64_t n,
                          const awe_patchy_consts* c, void* stream);

/* Binomial checkpoint schedule (host only, no device work) for a reverse sweep over
 * states S_1..S_{nsteps} with nslots restart slots.  Writes up to cap actions
 * (op, a, b) into actions[3*i..3*i+2] and the count into *count:
 *   op 0 ADVANCE  a -> b : run forward steps from state a to state b (b > a)
 *   op 1 STORE    slot a <- current state b
 *   op 2 RESTORE  current state <- slot a (which holds state b)
 *   op 3 REVERSE  adjoint step of level a (needs u^a: the current state is a or a + 1)
 * A state S_j = (u^j, u^{j-1}) holds two levels, so the reversals run in pairs: the state
 * reached for level j also serves level j - 1, and the binomial law places the checkpoints on
 * the pairs (for an even nsteps the fewest forward steps, for an odd one at most one more).
 * The first ADVANCE starts from the zero state S_0.  Returns INVALID_ARG if cap is too
 * small (*count then holds the needed size). */
awe_status awe_checkpoint_schedule(int32_t nsteps, int32_t nslots, int32_t* actions,
                                   int64_t cap, int64_t* count);

/* Tile-shape autotuner (setup call, synchronous).  The plan has a launch shape for its forward
 * solves (and Born modelling) and one for its adjoint steps (reverse sweeps and awe_adjoint); the
 * autotuner chooses each separately.  Candidates: 2D 8, 16, 24, 32 or 64 rows of 64 columns, and -
 * where the storage mode allows it - 8, 16, 24 or 32 rows with two time levels per launch (see
 * awe_plan_set_fusion); 3D 64 x {4, 8, 16} columns with z-blocks of the full depth, of 128, 64 or
 * 32 planes, and of the depth split evenly in 2 to 8 (rounded up to an even plane count).  The forward probe times the last probe_steps forward levels of the sweep (storing
 * the wavefield when the plan keeps one in FP32), the adjoint probe the last probe_steps adjoint
 * levels (with imaging when the plan keeps a wavefield; with PROBED storage both probes add to
 * the probe sums, taking their coefficients from the workspace), on the given inputs; the
 * fastest of each is kept for all later calls.  dd may be NULL (the adjoint probe then injects nothing).
 * Rebuilds the plan's device tables (the only allocation), overwrites the workspace and drops
 * any kept forward.  chosen (may be NULL) receives {tz, ty, bz} of the forward shape and the
 * fusion mode (awe_plan_get_tiles gives both shapes); best_ms (may be NULL) the sum of the two
 * winning probe times.
 * Result cache: when the environment variable AWE_TUNE_CACHE names a file, the call first looks
 * up a key made of the device (architecture name, compute units), the problem's shape (ndim,
 * shot count and a hash of every shot's grid, nt, receiver count and window), the storage, the
 * shot grouping and probe_steps.  A valid entry found there is put in effect without running
 * any probe (best_ms then returns the stored time); otherwise the probes run and the result is
 * added to the file.  The file is a JSON object with one entry per line,
 *   "key": {"fw": [tz, ty, bz], "rv": [tz, ty, bz], "fusion": f, "ms": t}
 * rewritten whole through a temporary file and a rename; lines of any other form are ignored
 * (and dropped at the next rewrite), and a file that cannot be written leaves the call's
 * result unaffected. */
awe_status awe_plan_autotune(awe_plan* plan, const float* m, const float* q, const float* dd,
                             int32_t probe_steps, void* ws, size_t ws_bytes, void* stream,
                             int32_t chosen[4], double* best_ms);

/* The launch shapes in effect: fwd / adj (each may be NULL) receive {tz, ty, bz} of the forward
 * solves and of the adjoint steps; fusion (may be NULL) the two-levels-per-launch mode. */
awe_status awe_plan_get_tiles(const awe_plan* plan, int32_t fwd[3], int32_t adj[3], int32_t* fusion);

/* Shot groups (batching, a12): the plan's shots, sorted by time offset, are split into
 * groups of consecutive shots; every call runs the time loop of one group after the other
 * (one launch per step covers the group's shots), so that a step's working set stays in the
 * 256 MB last-level cache.  ngroups = 0 (the default) chooses the count from the fields'
 * size (about 160 MB of three FP32 fields per group, at least 8 M points per group);
 * ngroups >= 1 forces that many (at most one per shot).  Results do not depend on the
 * grouping.  actual (may be NULL) receives the count in effect.  Rebuilds the device
 * tables and drops any kept forward.  Errors: INVALID_ARG, HIP. */
awe_status awe_plan_set_groups(awe_plan* plan, int32_t ngroups, int32_t* actual);

/* Set the tile shape explicitly (tz: 8, 12, 16, 20, 24, 32 or 64 rows in 2D; ty: 4, 8 or 16
 * rows and bz: z-block length, 0 = full depth, in 3D) of the forward solves and Born modelling
 * (dirs bit AWE_DIR_FORWARD), of the adjoint steps (AWE_DIR_ADJOINT) or of both;
 * awe_plan_set_tiles sets both.  Results do not depend on the tile shapes (every point's
 * arithmetic and every sum's order are fixed).  Rebuilds the device tables of the directions
 * set. */
enum { AWE_DIR_FORWARD = 1, AWE_DIR_ADJOINT = 2, AWE_DIR_BOTH = 3 };
awe_status awe_plan_set_tiles_dir(awe_plan* plan, int32_t dirs, int32_t tz, int32_t ty, int32_t bz);
awe_status awe_plan_set_tiles(awe_plan* plan, int32_t tz, int32_t ty, int32_t bz);

/* 2D only: advance two time levels per launch, chosen per direction by the bits of mode:
 * AWE_FUSE_FORWARD for forward solves and Born modelling, AWE_FUSE_ADJOINT for reverse sweeps (0, the default:
 * one level per launch everywhere).  The two-level kernels serve forward solves without
 * storage, with FULL FP32 storage or into PROBED sums, reverse sweeps from FULL FP32
 * storage, into PROBED sums or without imaging, and the paired reversals of a CHECKPOINT
 * gradient (imaging from the recomputed forward levels); other modes always use one level per
 * launch.
 * Results are bitwise identical either way (a two-level launch adds both levels' terms to an
 * FP64 sum in the order two launches would).  Two levels per launch need tiles of 8, 16, 24 or 32 rows (16 or 32 are set
 * otherwise).  Errors: INVALID_ARG (mode outside 0..3), HIP. */
enum { AWE_FUSE_NONE = 0, AWE_FUSE_FORWARD = 1, AWE_FUSE_ADJOINT = 2, AWE_FUSE_BOTH = 3 };
awe_status awe_plan_set_fusion(awe_plan* plan, int32_t mode);

/* Kernel timing (measurement aid).  After awe_profile_enable, every stride-th time-step
 * launch of the compute calls on this plan is bracketed by a pair of HIP events recorded on
 * the call's stream, for up to max_launches timed intervals; further launches are not timed.
 * The steps of one sweep (the forward or the adjoint step loop of a call, per shot group) and
 * the forward steps of one checkpoint advance each form one interval, which counts every launch
 * it holds, so that no event is recorded between them; other step launches are timed one by
 * one.
 * The records are stream work, so they are also captured into a HIP graph and then time
 * the graph's replays.  Classes: 0 forward step, 1 adjoint step (with imaging and, in 3D,
 * receiver injection), 2 Born step.  awe_profile_read waits for the recorded events,
 * returns per class the number of timed launches and the summed time of their intervals in ms,
 * and restarts the count.  Enabling creates HIP events (host resources, no device memory). */
awe_status awe_profile_enable(awe_plan* plan, int64_t max_launches, int32_t stride);
awe_status awe_profile_read(awe_plan* plan, int64_t counts[3], double ms[3]);
awe_status awe_profile_disable(awe_plan* plan);

const char* awe_status_string(awe_status s);
const char* awe_last_error(void);
int awe_version(void);

#ifdef __cplusplus
}
#endif
#endif /* AWE_H */
