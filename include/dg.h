/*
 * dg.h — C ABI of the MI355X nodal discontinuous-Galerkin right-hand-side library.
 *
 * The library evaluates the nodal DG semi-discretisation of the compressible
 * Euler equations on affine tetrahedra and advances it with low-storage RK4:
 * the per-element arrays of nodal unknowns the paper describes (Sec. 1,
 * Fig. "dg_mesh"), the periodic isentropic-vortex Euler/RK4 benchmark of
 * Sec. 5.2, and the bandwidth-bound low-order element kernels profiled in
 * Sec. 5.4.  The paper prints no DG formula; the operations below follow the
 * textbook nodal DG method (Hesthaven & Warburton), as stated per entry point.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every call returns a dg_status; DG_OK is 0.  On failure a message is
 *    available from dg_last_error() (thread-local, valid until the next call
 *    on the same thread).  No C++ exception crosses this interface.
 *  - State layout (field-major): q[nf][E][Np] FP64, contiguous, element e's
 *    node i of field f at q[(f * E + e) * Np + i].  nf = 5 for Euler:
 *    (rho, rho u, rho v, rho w, E_total).
 *  - Node order inside an element: the equidistant lattice of order p walked
 *    with t outermost, then s, then r innermost, each point moved by the
 *    warp & blend map (Warburton 2006) and keeping its index.  Reference
 *    vertices v1=(-1,-1,-1), v2=(1,-1,-1), v3=(-1,1,-1), v4=(-1,-1,1); faces
 *    f0={t=-1}, f1={s=-1}, f2={r+s+t=-1}, f3={r=-1}.
 *  - Device buffers (q, rhs, work) are caller-owned device memory, 8-byte
 *    aligned at least (256-byte recommended; at p = 1 and 3 a 16-byte-aligned
 *    state lets the element kernels copy it into LDS by DMA, with the same
 *    results); the library never frees them and keeps no pointer past return.  Compute calls are asynchronous on the given
 *    HIP stream (0 = the null stream); argument checks are synchronous.
 *  - Handles (dg_mesh, dg_thermo, dg_mech, dg_mlp, dg_batch) own their tables;
 *    *_destroy frees them.
 *    A handle is immutable after creation, so calls on different streams may
 *    share it.
 */
#ifndef DG_H
#define DG_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DG_OK = 0,
  DG_ERR_ARG = 1,         /* null/misaligned pointer, size or enum out of range */
  DG_ERR_MESH = 2,        /* non-positive Jacobian, unmatched or over-shared face */
  DG_ERR_ALLOC = 3,       /* device or host allocation failed */
  DG_ERR_HIP = 4,         /* a HIP runtime call failed (message carries its text) */
  DG_ERR_NOCONV = 5,      /* iterative solve did not converge */
  DG_ERR_NONFINITE = 6,   /* non-finite value detected */
  DG_ERR_UNSUPPORTED = 7  /* valid request the library does not implement */
} dg_status;

/* Precision of the element-local contractions (volume divergence and lift)
 * only; pointwise fluxes, the face flux, the state and the RK update are FP64
 * in every mode. */
typedef enum { DG_FP64 = 0, DG_FP32 = 1, DG_SPLIT_BF16 = 2 } dg_precision;

struct dg_thermo_s;
struct dg_mech_s;

typedef struct {
  int model;      /* 0 = Euler (ideal gas), 1 = reacting Navier-Stokes */
  double gamma;   /* Euler: ratio of specific heats, > 1 (unused by model 1) */
  double mu, Pr, Sc;                 /* model 1: viscosity [Pa s] >= 0, Prandtl and Schmidt numbers > 0 */
  const struct dg_thermo_s* thermo;  /* model 1: species thermodynamics (7 species), required */
  const struct dg_mech_s* mech;      /* model 1: reactions; NULL = no chemical sources */
  /* model 1 through dg_rhs / dg_rk_step: caller-owned device scratch for the
   * temperatures, Newton counts and lifted gradients (dg_rhs: at least
   * DG_NS_RHS_WORK E Np doubles; dg_rk_step: DG_NS_STEP_WORK E Np), and the
   * Newton tolerance [K] and step limit (<= 0 selects 1e-10 and 50).  The
   * temperature solve starts from 1000 K.  Unused by model 0. */
  double* work;
  double tol;
  int max_iter;
} dg_params;
#define DG_NS_RHS_WORK 35  /* T (1), Newton counts (1), lifted gradients (33) per node */
#define DG_NS_STEP_WORK 59 /* T (1) + the dg_ns_rk_step scratch (58) per node */

typedef struct dg_mesh_s* dg_mesh;

/* Reference-element tables of order p (1..4), computed on the host (no GPU
 * needed).  Nodes and operators of the nodal basis as defined above:
 *   rst   [Np][3]        node coordinates (r, s, t)
 *   Dr,Ds,Dt [Np][Np]    Dr[i][j] = d l_j/dr at node i (row-major)
 *   LIFT  [Np][4*Nfp]    M^{-1} E, columns face-major (f, m)
 *   Fmask [4][Nfp]       ascending node indices on each face
 * Any output pointer may be NULL.  Returns DG_ERR_ARG for p outside 1..4. */
dg_status dg_reference_operators(int order, double* rst, double* Dr, double* Ds, double* Dt,
                                 double* LIFT, int32_t* Fmask);

/* Build a mesh handle on `device` from affine tetrahedra.
 *   elem_xyz  host [n_elem][4][3]  vertex coordinates (periodic images given
 *                                  unwrapped); the reference-to-physical map
 *                                  x = -(1+r+s+t)/2 X1 + (1+r)/2 X2 + (1+s)/2 X3
 *                                  + (1+t)/2 X4 must have J > 0
 *   elem_vid  host [n_elem][4]     global vertex ids; faces match on the
 *                                  sorted id triple, so periodic images must
 *                                  share ids; every face must occur exactly twice
 * Geometric factors, face connectivity (neighbour, neighbour face and vertex
 * permutation per face) and the reference operators are computed on the host
 * and copied to the device (synchronous).  Errors: DG_ERR_ARG (order not in
 * 1..4, n_elem < 1 or > 2^27, null pointers, bad device), DG_ERR_MESH (J <= 0,
 * unmatched face), DG_ERR_ALLOC / DG_ERR_HIP. */
dg_status dg_mesh_create(int order, int64_t n_elem, const double* elem_xyz, const int64_t* elem_vid,
                         int device, dg_mesh* out);
dg_status dg_mesh_info(dg_mesh m, int64_t* n_elem, int* np, int* nfp);
/* Physical node coordinates, host [n_elem][Np][3] (parity hook). */
dg_status dg_mesh_nodes(dg_mesh m, double* xyz_host);
/* Face-node map as seen by the library, host [n_elem][4*Nfp] each: neighbour
 * element and neighbour volume-node index of every face node (parity hook). */
dg_status dg_mesh_face_map(dg_mesh m, int64_t* nbr_elem, int32_t* nbr_node);
dg_status dg_mesh_destroy(dg_mesh m);

/* Strong-form nodal DG right-hand side (the Euler benchmark of Sec. 5.2; the
 * reacting flow of Sec. 5 with model 1).  Model 0, Euler:
 *   rhs = -sum_{a=r,s,t} D_a (sum_d da/dx_d F_d(q))
 *         + LIFT * ( Fscale * [ 1/2 n.(F(q-) - F(q+)) - 1/2 lam (q- - q+) ] )
 * with the local Lax-Friedrichs speed lam = max(|u-.n| + c-, |u+.n| + c+) at
 * every face node.  q, rhs: device [5][E][Np] FP64 (must not alias).
 * prec selects the contraction precision: DG_FP64; DG_FP32 (operator and
 * operands rounded to FP32, FP32 accumulation); DG_SPLIT_BF16 (x = hi + lo
 * with hi = bf16(fp32(x)), lo = bf16(fp32(x) - hi), Op X ~ Op_hi X_hi +
 * Op_hi X_lo + Op_lo X_hi accumulated in FP32).  Fluxes, jumps and the
 * result are FP64 in every mode.  Model 1, reacting Navier-Stokes (the
 * equations of dg_ns_rhs below): q, rhs device [12][E][Np]; the temperature
 * Newton solve (from 1000 K), the lifted gradients and the right-hand side
 * with sources run in prm->work; DG_FP64 only (other precisions return
 * DG_ERR_UNSUPPORTED).  A non-finite result raises the device's non-finite
 * flag (dg_synchronize).  Asynchronous on `stream`. */
dg_status dg_rhs(dg_mesh m, const dg_params* prm, dg_precision prec, const double* q, double* rhs,
                 hipStream_t stream);

/* One step of Carpenter & Kennedy's five-stage fourth-order 2N-storage
 * Runge-Kutta scheme (the paper's explicit RK4, Sec. 5.2, read as the
 * low-storage form):  res <- 0; for s = 1..5: res <- a_s res + dt RHS(q);
 * q <- q + b_s res.  q: device [5][E][Np], updated in place.  work: device
 * scratch of at least 2 * 5 * E * Np doubles, caller-owned, contents
 * overwritten.  Model 1 (reacting Navier-Stokes, DG_FP64 only): q is
 * [12][E][Np], work is unused and prm->work (DG_NS_STEP_WORK E Np doubles)
 * holds the temperatures, whose solve starts from 1000 K at the first stage
 * and from the previous stage's values after it (as dg_ns_rk_step).  A
 * non-finite new state raises the device's non-finite flag.  t is accepted for non-autonomous models (the Euler RHS does
 * not depend on it).  With the mesh's launch configuration for prec (below)
 * each stage is one fused launch (RHS + stage update into another state
 * buffer: the intermediate states and the residual rotate through q and
 * the two halves of work so that the fifth stage writes q, with no copy)
 * or an RHS launch into work followed by the pointwise update of q in
 * place; both give the same bits. */
dg_status dg_rk_step(dg_mesh m, const dg_params* prm, dg_precision prec, double* q, double* work,
                     double t, double dt, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * Euler step as dg_rk_step (model 0, any contraction precision, the mesh's
 * launch configuration, the same kernels and so the same bits), with the
 * two state-sized work buffers in a fixed array the library holds
 * on each GPU instead of a caller workspace.  It calls no allocator.
 *  - Limit: the state may hold at most DG_NOALLOC_MAX_STATE doubles
 *    (5 E Np <= 8,388,608: up to 83,886 tets at p = 3, e.g. one GPU's
 *    82,944-tet share of the 48^3 mesh split over eight GPUs); larger
 *    states return DG_ERR_ARG.  The array takes 2 x 64 MiB of every GPU
 *    the library runs on, until the process ends.
 *  - Every call on one GPU uses that GPU's one array: calls that overlap in
 *    time on one GPU (different streams or threads) race and must be
 *    serialised by the caller.  Nothing in the array needs clearing between
 *    calls (the first stage does not read the old residual).
 *  - model 1 returns DG_ERR_UNSUPPORTED. */
#define DG_NOALLOC_MAX_STATE (8u << 20)
dg_status dg_rk_step_noalloc(dg_mesh m, const dg_params* prm, dg_precision prec, double* q, double t, double dt,
                             hipStream_t stream);

/* Launch configuration of one mesh's RHS and Runge-Kutta kernels for one
 * contraction precision.  Results do not depend on it (bitwise). */
typedef struct {
  int waves_per_block; /* 16-element tiles per block: 2 or 4 up to p = 3.  At
                          p = 4 the FP64 kernel runs 2 and the FP32 / split
                          BF16 kernels 1, whatever is requested. */
  int rk_fused;        /* 1 = fused stage launches, 0 = RHS launch + update */
  int lds_stage;       /* 1 = stage the state tile into LDS by direct
                          global-to-LDS loads where that path exists (FP64
                          and FP32 contractions, Np a multiple of 4, q
                          16-byte aligned), 0 = through registers */
  int xcd_run;         /* single-mesh RHS and stage kernels (the batch
                          ignores it): workgroups are dispatched round-robin
                          to the 8 XCDs (each with its own L2); with
                          xcd_run = k > 1 each XCD takes runs of k
                          consecutive blocks of tiles, all XCDs still
                          sweeping the mesh together, so that neighbouring
                          tiles share an L2.  1 .. 64; 1 = plain order */
} dg_launch_config;
/* Initial configuration of every precision: {4, 1, 1, 1}.  Set and get are
 * synchronous host calls that must not overlap calls running on the mesh. */
dg_status dg_mesh_set_launch(dg_mesh m, dg_precision prec, const dg_launch_config* cfg);
dg_status dg_mesh_get_launch(dg_mesh m, dg_precision prec, dg_launch_config* cfg);
/* Times every launch configuration of the mesh at precision prec (`trials`
 * dg_rk_step calls each after one warm-up, on a uniform state in temporary
 * device buffers the call allocates and frees), keeps the fastest and sets
 * it.  With cache_path != NULL the choice is first looked up in that JSON
 * file under a key of (device architecture, CU count, precision, p, E) and,
 * when tuned, written back.  chosen (may be NULL) receives the
 * configuration, best_ms (may be NULL) its time per step, negative when it
 * came from the cache.  Synchronous on `stream`; must not overlap other calls
 * on the mesh. */
dg_status dg_autotune(dg_mesh m, const dg_params* prm, dg_precision prec, const char* cache_path, int trials,
                      dg_launch_config* chosen, double* best_ms, hipStream_t stream);

/* Pointwise stage update used by unfused stepping:
 *   res <- a * res + dt * rhs;  q <- q + b * res   over n doubles. */
dg_status dg_lsrk_update(int64_t n, double a, double b, double dt, const double* rhs, double* res,
                         double* q, hipStream_t stream);

/* ---- reacting flow: species thermodynamics, temperature, sources -------- */
/* State of a reacting mixture: q[5 + ns][n] FP64 field-major (n points),
 * fields (rho, rho u, rho v, rho w, E_total, rho Y_1 .. rho Y_ns), SI units. */

typedef struct dg_thermo_s* dg_thermo;
typedef struct dg_mech_s* dg_mech;

/* Species table for temperature-dependent thermodynamics (the paper's
 * multispecies reacting flow, Sec. 5; one-range polynomial reading):
 * R_k = R_u / W_k, cp_k/R_k = a1 + a2 T + a3 T^2 + a4 T^3 + a5 T^4,
 * h_k/R_k = a1 T + a2 T^2/2 + a3 T^3/3 + a4 T^4/4 + a5 T^5/5 + a6, e_k = h_k - R_k T.
 *   W       host [ns]     molar masses, kg/mol, > 0
 *   coeffs  host [ns][6]  (a1 .. a6), a6 in K
 * ns in 1..8.  The handle keeps a host copy (passed to kernels by value). */
dg_status dg_thermo_create(int n_species, const double* W, const double* coeffs, int device, dg_thermo* out);
dg_status dg_thermo_destroy(dg_thermo th);

/* Irreversible Arrhenius mechanism over the species of `th`:
 * k_j = A_j exp(-Ea_j / (R_u T)), r_j = k_j prod_k C_k^{nu'_kj}, C_k = rho Y_k / W_k,
 * omega_k = W_k sum_j (nu''_kj - nu'_kj) r_j  [kg / (m^3 s)].
 *   A, Ea       host [nr]      (SI: mol, m^3, s; J/mol), A >= 0
 *   nu_r, nu_p  host [nr][ns]  reactant / product coefficients, integers 0..3
 * nr in 1..8. */
dg_status dg_mech_create(dg_thermo th, int n_reactions, const double* A, const double* Ea, const int32_t* nu_r,
                         const int32_t* nu_p, dg_mech* out);
dg_status dg_mech_destroy(dg_mech m);

struct dg_mlp_s;

/* Temperature from the conserved state by Newton's method on
 * e(T; Y) = E/rho - |m|^2/(2 rho^2):  T <- T - (e(T) - e) / cv(T),
 * cv = sum Y_k (cp_k - R_k), iterates clamped to [100, 6000] K, stopping when
 * |T_{n+1} - T_n| < tol (temperature-dependent thermochemistry of the
 * reacting flow, Sec. 4 and 5).  q: device [5+ns][n]; T_guess: device [n]
 * initial iterates, or NULL to start every point at 1000 K; T_out: device
 * [n]; iters: device int32 [n], the step count, or -1 where max_iter steps did
 * not converge (T_out then holds the last iterate).  A step cut by the clamp
 * is never convergence, so a point whose root lies outside [100, 6000] K
 * reports -1; a point whose state is not finite ends at once with -1 and a
 * non-finite T.  Either failure raises the device's no-convergence or
 * non-finite flag, which the next dg_synchronize returns as DG_ERR_NOCONV /
 * DG_ERR_NONFINITE.  guess: a learned-guess network (see dg_mlp_*) or NULL;
 * with it, T_guess must be NULL and the solve is that of
 * dg_temperature_learned with at most 8 steps from the network's clamped
 * prediction, then a restart from 1000 K.  Asynchronous on `stream`. */
dg_status dg_temperature(int64_t n, const double* q, const double* T_guess, double* T_out, int32_t* iters,
                         dg_thermo th, double tol, int max_iter, const struct dg_mlp_s* guess, hipStream_t stream);

/* Species mass sources omega: device [ns][n] from q (device [5+ns][n]) and
 * T (device [n]); the rates of dg_mech_create.  Asynchronous on `stream`. */
dg_status dg_sources(int64_t n, const double* q, const double* T, double* omega, dg_mech mech, hipStream_t stream);

/* Waits for `stream` on `device`, then reads and clears the device's failure
 * flags: DG_ERR_NONFINITE if a kernel since the last call produced a
 * non-finite state, right-hand side or temperature, else DG_ERR_NOCONV if a
 * Newton solve ended with iteration count -1, else DG_OK.  The flags are one
 * word per device shared by every stream and handle on it: a failure on any
 * stream is reported by the next dg_synchronize on that device. */
dg_status dg_synchronize(int device, hipStream_t stream);

/* ---- learned temperature guess ------------------------------------------ */
/* Multilayer perceptron x -> T0 with widths 9 -> 64 -> 64 -> 64 -> 1 and tanh
 * (9,025 parameters), x = standardised (log rho, e, Y_1 .. Y_7).  BF16 operands
 * on the matrix cores with FP32 accumulation; bias and tanh in FP32,
 * activations rounded to BF16; FP32 master weights and Adam moments.
 * Parameter vector (host FP32 [9025]): W1[64][9], b1[64], W2[64][64], b2[64],
 * W3[64][64], b3[64], W4[1][64], b4[1].  Training data are columns of a
 * reacting state q (device [12][ld]) selected by idx (device int64 [batch])
 * with targets T (device [ld]).  A handle's scratch and Adam state are shared
 * by every call on it: calls on one handle must not overlap. */
typedef struct dg_mlp_s* dg_mlp;

/* Glorot-uniform weights (seeded), zero biases, identity normalisation. */
dg_status dg_mlp_create(int device, uint64_t seed, dg_mlp* out);
dg_status dg_mlp_destroy(dg_mlp m);
/* Replace / read the FP32 master parameters (set also clears Adam state). */
dg_status dg_mlp_set_params(dg_mlp m, const float* params);
dg_status dg_mlp_get_params(dg_mlp m, float* params);
/* Feature means / standard deviations (host [9]) and target mean / std. */
dg_status dg_mlp_set_normalization(dg_mlp m, const double* feat_mean, const double* feat_std, double T_mean,
                                   double T_std);
dg_status dg_mlp_get_normalization(dg_mlp m, double* feat_mean, double* feat_std, double* T_mean, double* T_std);
/* Normalisation fitted on the samples idx[0..n) (synchronous); a feature whose
 * standard deviation is below 1e-6 max(|mean|, 1) is centred, not scaled. */
dg_status dg_mlp_fit_normalization(dg_mlp m, int64_t n, int64_t ld, const double* q, const int64_t* idx,
                                   const double* T);
/* MSE loss mean((out - (T - T_mean)/T_std)^2) over the batch and its gradient
 * (device FP32 [9025] in parameter order); either output may be NULL. */
dg_status dg_mlp_loss_grad(dg_mlp m, int64_t batch, int64_t ld, const double* q, const int64_t* idx,
                           const double* T, float* grad, float* loss, hipStream_t stream);
/* One Adam step (betas 0.9 / 0.999, eps 1e-8, bias-corrected) on that gradient. */
dg_status dg_mlp_train_step(dg_mlp m, int64_t batch, int64_t ld, const double* q, const int64_t* idx,
                            const double* T, float lr, float* loss, hipStream_t stream);
/* Predicted temperature (de-standardised, unclamped) of columns 0..n of q. */
dg_status dg_mlp_predict(dg_mlp m, int64_t n, int64_t ld, const double* q, double* T_pred, hipStream_t stream);
/* dg_temperature started from the clamped prediction: at most
 * learned_max_iter Newton steps, then, where not converged, a restart from
 * T_default with max_iter steps (counted in *fallback_count, device int32,
 * may be NULL).  iters = total steps, -1 if the restart fails too.  The
 * answer is the same converged root the plain solve finds.  ns must be 7. */
dg_status dg_temperature_learned(dg_thermo th, dg_mlp m, int64_t n, const double* q, double T_default,
                                 double* T_out, int32_t* iters, double tol, int max_iter, int learned_max_iter,
                                 int32_t* fallback_count, hipStream_t stream);

/* ---- reacting Navier-Stokes with BR1 viscous terms ---------------------- */
/* Viscous, multispecies, reacting flow as named for MIRGE-Com (Sec. 5); the
 * paper prints no equation, so the textbook forms are used.  State
 * q[12][E][Np] (rho, rho u, rho v, rho w, E_total, rho Y_1 .. rho Y_7) with
 * temperatures T[E][Np] from dg_temperature; p = rho R_mix T.  Viscous
 * terms by Bassi & Rebay's first scheme: lifted gradients of
 * v = (u, v, w, T, Y_1 .. Y_7) with the central trace,
 *   sigma_d(v) = sum_a (da/dx_d) D_a v + LIFT( Fscale n_d (v+ - v-) / 2 ),
 * stored node-major as sigma[E][Np][3 c + d]; stress tau = mu (grad u + grad u^T
 * - 2/3 div u I), heat flux -kappa grad T with kappa = mu cp / Pr, species
 * flux J_k = -(mu / Sc) grad Y_k; viscous flux (0, tau, u.tau + kappa grad T
 * - sum_k h_k J_k, -J_k).  Total flux F = F_inviscid - F_viscous; surface
 * flux: local Lax-Friedrichs on the inviscid part (sound speed from
 * gamma_mix = cp / cv), central average on the viscous part, no penalty:
 *   rhs = -sum_a D_a (sum_d da/dx_d F_d) + LIFT( Fscale [ n.(F- - F+) / 2
 *         - lam (q- - q+) / 2 ] ) + (0, 0, 0, 0, 0, omega_1 .. omega_7),
 * omega from dg_sources when prm->mech is set.  prm->model must be 1 and
 * prm->thermo (and mech, if given) must hold 7 species on the mesh's device.
 * Errors: DG_ERR_ARG for bad parameters, pointers or aliasing,
 * DG_ERR_UNSUPPORTED for a species count other than 7. */

/* sigma (device [E][Np][33]) receives the lifted gradients; rhs (device
 * [12][E][Np]) the right-hand side.  q, T, sigma and rhs must not overlap. */
dg_status dg_ns_rhs(dg_mesh m, const dg_params* prm, const double* q, const double* T, double* sigma, double* rhs,
                    hipStream_t stream);
/* One LSRK(5,4) step of the reacting NS system, each stage: temperature
 * Newton (started from T, tolerance tol, at most max_iter steps), gradient
 * pass, right-hand side fused with the stage update.  q (device
 * [12][E][Np]) is updated in place; T (device [E][Np]) is the first stage's
 * Newton start and returns the temperatures of the last stage's input.
 * work: device scratch of 58 E Np doubles (two state-sized buffers that the
 * residual and the intermediate states rotate through, as in dg_rk_step;
 * gradients; the last E Np doubles hold the last stage's int32 Newton
 * iteration counts, -1 where it did not converge). */
dg_status dg_ns_rk_step(dg_mesh m, const dg_params* prm, double* q, double* T, double* work, double dt, double tol,
                        int max_iter, hipStream_t stream);

/* ---- batched stepping of many meshes ------------------------------------ */
/* A batch advances many independent meshes of mixed order (p = 1..4) and
 * size with a few kernel launches per Runge-Kutta stage: a work list holds
 * one item per (mesh, 16-element tile) of every mesh.  In the mixed mode one
 * persistent kernel per stage walks the whole list, running each item with
 * its mesh's order; in the per-order modes one kernel per order present and
 * stage walks that order's items (the chains of different orders either
 * concurrent on forked streams, or in sequence on one stream).  This is the launch counterpart of
 * concatenating independent calls into one larger call (Sec. 4.2,
 * "Concatenation of Function Calls"), aimed at the per-launch floor that
 * small meshes hit (Sec. 5.2, MIRGE-Com vs. MFEM).  Each mesh's result is
 * bitwise the one dg_rk_step gives it alone at the same precision, because
 * both modes run the same tile routine.  Contractions are DG_FP32 or
 * DG_SPLIT_BF16 (DG_FP64 returns DG_ERR_UNSUPPORTED); the state and stage
 * update are FP64.  A batch keeps pointers to the bound caller buffers (and,
 * once a step was run with use_graph, a captured graph that holds them): they
 * must stay valid until the next bind or destroy.  Calls on one batch must
 * not overlap. */
typedef struct dg_batch_s* dg_batch;

/* Launch shape of the batched stage kernels. */
typedef struct {
  int waves_per_block; /* 2, 4 or 8 (64 lanes each) */
  int blocks_per_cu;   /* 1..4, capped by the kernel's occupancy */
  int order;           /* work-list order: 0 = highest order first, 1 = mesh order */
  int xcd_chunks;      /* 1 = each of the 8 XCDs walks a contiguous eighth of the
                          list, 0 = the whole grid strides over the list */
  int per_order;       /* 0 = one mixed-order launch per stage; 1 = one
                          launch per order present and stage, each order's
                          chain on a stream of its own (forked and joined);
                          2 = the same launches on one stream, stage by
                          stage.  With 1 or 2 the four fields above are
                          unused: each order's kernel has its own fixed shape */
} dg_batch_config;

/* Meshes (n >= 1, all on the same device, not freed while the batch lives)
 * and the contraction precision.  Builds and uploads the work lists; the
 * initial launch shape is {4, 2, 0, 0, 1}. */
dg_status dg_batch_create(const dg_mesh* meshes, int n, dg_precision prec, dg_batch* out);
dg_status dg_batch_destroy(dg_batch b);
/* Bind the state of every mesh: q[i] device [5][E_i][Np_i] (updated in
 * place by each step), work[i] device scratch of 2 * 5 * E_i * Np_i doubles
 * (not overlapping q[i]), dt device [n] time steps (read by every step, so
 * the caller may change them between steps).  q and work are host arrays of n
 * device pointers.  Drops a captured graph.  Synchronous. */
dg_status dg_batch_bind(dg_batch b, double* const* q, double* const* work, const double* dt);
dg_status dg_batch_set_config(dg_batch b, const dg_batch_config* cfg);
dg_status dg_batch_get_config(dg_batch b, dg_batch_config* cfg);
/* One LSRK(5,4) step of every bound mesh: five stage launches and one copy
 * launch (per order present in the per-order modes).  use_graph != 0 replays
 * a graph of those launches on `stream`, capturing it first when none
 * matches the current binding, configuration and gamma; use_graph == 0
 * launches them directly (forking to the batch's own streams and joining
 * back into `stream` when per_order == 1). */
dg_status dg_batch_rk_step(dg_batch b, const dg_params* prm, int use_graph, hipStream_t stream);
/* Work items, total elements, and kernel nodes of the captured graph (0 when
 * none is held).  Any pointer may be NULL. */
dg_status dg_batch_info(dg_batch b, int64_t* n_items, int64_t* n_elem, int* graph_kernel_nodes);
/* Time every candidate launch shape (both per-order modes, and the mixed mode
 * at waves_per_block x blocks_per_cu x order x xcd_chunks) with `trials`
 * steps each after one warm-up step on the bound
 * buffers, keep the fastest and set it.  The bound q are saved before and
 * restored after (a temporary device copy), so tuning leaves the state as it
 * was; work is overwritten.  With cache_path != NULL the choice is looked up
 * first in that JSON file under a key of (device, precision, multiset of
 * (p, E)) and, when tuned, written back.  chosen (may be NULL) receives the
 * shape; best_ms (may be NULL) its time per step (negative when taken from
 * the cache without timing).  Synchronous on `stream`. */
dg_status dg_batch_autotune(dg_batch b, const dg_params* prm, const char* cache_path, int trials,
                            dg_batch_config* chosen, double* best_ms, hipStream_t stream);

const char* dg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DG_H */
