/*
 * dg_hex.h — C ABI of the tensor-product hexahedron path of the MI355X nodal
 * DG library: the element of the paper's own Euler benchmarks (Sec. 5.2:
 * the p = 4 isentropic vortex and the p = 1 case on tensor-product
 * elements), on periodic rectilinear grids.
 *
 * Conventions are those of dg.h (status codes, dg_last_error, caller-owned
 * device buffers, asynchronous calls on the given stream, synchronous
 * argument checks, the failure flag read by dg_synchronize).
 *
 * Mesh: nx x ny x nz cells; cell (i, j, k) is the axis-aligned box
 * [gx[i], gx[i+1]] x [gy[j], gy[j+1]] x [gz[k], gz[k+1]], element id
 * e = i + nx (j + ny k); the grid is periodic in every direction (cell
 * nx - 1 neighbours cell 0; gx[nx] - gx[0] is the period).
 * Element: tensor product of the p + 1 Legendre-Gauss-Lobatto points,
 * node (a, b, c) at reference (r_a, s_b, t_c) with index
 * a + (p + 1)(b + (p + 1) c); physical x = gx[i] + (1 + r_a)(gx[i+1] - gx[i]) / 2.
 * State layout: q[5][E][Np] FP64, Np = (p + 1)^3, fields as in dg.h.
 */
#ifndef DG_HEX_H
#define DG_HEX_H

#include "dg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg_hex_mesh_s* dg_hex_mesh;

/* Host tables of the order-p element (1 <= order <= 4), any output may be
 * NULL: x [p+1] LGL points; D1 [p+1][p+1] row-major, D1[i][j] = l_j'(x_i)
 * (l_j the Lagrange polynomials on the points); lift [p+1][2] row-major, the
 * columns M1^{-1} e_0 and M1^{-1} e_p of the exact 1-D mass matrix
 * M1[i][j] = int_{-1}^{1} l_i l_j.  The values are the exact ones at the
 * FP64 points, rounded once.  DG_ERR_ARG for other orders. */
dg_status dg_hex_reference_operators(int order, double* x, double* D1, double* lift);

/* Builds the mesh on `device` from the host grid lines gx [nx+1], gy [ny+1],
 * gz [nz+1] (copied), which must increase strictly (else DG_ERR_MESH); at
 * most 2^31 - 1 nodes (E Np).  Synchronous; *out owns its device tables (2 / h per cell
 * and axis, the 1-D operators). */
dg_status dg_hex_mesh_create(int order, int nx, int ny, int nz, const double* gx, const double* gy,
                             const double* gz, int device, dg_hex_mesh* out);
dg_status dg_hex_mesh_info(dg_hex_mesh m, int64_t* n_elem, int* np);
/* Physical node coordinates, host [E][Np][3]. */
dg_status dg_hex_mesh_nodes(dg_hex_mesh m, double* xyz);
dg_status dg_hex_mesh_destroy(dg_hex_mesh m);

/* Strong-form Euler right-hand side (model 0 of dg_params; gamma > 1), FP64,
 * of the nodal DG method on the hexahedra:
 *   rhs = - sum_d (2 / h_d) D_d F_d + sum_faces (2 / h_d) l_side x Delta,
 *   Delta = 1/2 n.(F(q-) - F(q+)) - 1/2 lam (q- - q+),
 *   lam = max(|u-.n| + c-, |u+.n| + c+)   (local Lax-Friedrichs),
 * D_d the 1-D derivative along direction d (sum factorisation) and l_side
 * the lift column of the face's side, acting along the lines normal to the
 * face.  q and rhs: device [5][E][Np], must not overlap.  model 1 returns
 * DG_ERR_UNSUPPORTED. */
dg_status dg_hex_rhs(dg_hex_mesh m, const dg_params* prm, const double* q, double* rhs, hipStream_t stream);

/* One LSRK(5,4) step (Carpenter & Kennedy 1994, as dg_rk_step), q in place;
 * work: device, at least 2 x 5 E Np doubles, not overlapping q. */
dg_status dg_hex_rk_step(dg_hex_mesh m, const dg_params* prm, double* q, double* work, double t, double dt,
                         hipStream_t stream);

/* Overintegrated form (the paper names overintegration among what its
 * shock cases need, Sec. 5.3): the weak form of the same method,
 *   (M rhs)_i = int_K grad l_i . F(q_h) - int_dK l_i Fhat,
 *   Fhat = 1/2 n.(F(q-) + F(q+)) + 1/2 lam (q- - q+),
 * with the nodal interpolant q_h, the fluxes and Fhat evaluated at
 * nq = ceil(3 (p + 1) / 2) Gauss-Legendre points per direction (the "3/2
 * rule" against the aliasing of quadratic nonlinearities).  It factors into
 * rectangular 1-D contractions: B[k][j] = l_j(xi_k) (nq x (p+1)) to the
 * quadrature points, and S = M1^{-1} B'^T W, P = M1^{-1} B^T W ((p+1) x nq)
 * back to the nodes:
 *   rhs = sum_d (2 / h_d) [ (S along d, P along the others) F_d(quad)
 *                           - sum_side l_side x (P x P) Fhat_face(quad) ].
 * Host tables for tests (any output may be NULL): *nq, the Gauss points
 * xq [nq] and weights wq [nq] (correctly rounded), and tables =
 * [B (nq x (p+1)) | S ((p+1) x nq) | P ((p+1) x nq) | lift ((p+1) x 2)],
 * row-major, exact at the FP64 points and weights and rounded once. */
dg_status dg_hex_oi_operators(int order, int* nq, double* xq, double* wq, double* tables);
/* The overintegrated right-hand side and LSRK step; arguments and rules as
 * dg_hex_rhs / dg_hex_rk_step. */
dg_status dg_hex_rhs_oi(dg_hex_mesh m, const dg_params* prm, const double* q, double* rhs, hipStream_t stream);
dg_status dg_hex_rk_step_oi(dg_hex_mesh m, const dg_params* prm, double* q, double* work, double t, double dt,
                            hipStream_t stream);

/* Shock capturing (the paper names artificial viscosity and shock limiting
 * among what its shock cases need, Sec. 5.3; the formulas below are the
 * readings this library implements):
 *  - indicator per element (Persson & Peraire 2006): the density's
 *    coefficients c in the orthonormal tensor Legendre basis, S = (energy of
 *    the modes with max(i, j, k) = p) / (total energy), s = log10 S
 *    (-inf for S = 0);
 *  - viscosity per element eps = c_eps h / p max(|u| + c) ramp(s), h the
 *    element's smallest edge, ramp 0 below s0 - kappa, 1 above s0 + kappa,
 *    (1 + sin(pi (s - s0) / (2 kappa))) / 2 between;
 *  - d q/dt += div(eps grad q) for every conserved field, BR1 with central
 *    fluxes: sigma_d = (2/h_d)(D_d q + sum_side l_side n_d (q+ - q-)/2),
 *    G_d = eps sigma_d, added as sum_d (2/h_d)(D_d G_d + sum_side l_side
 *    n_d (G_d+ - G_d-)/2);
 *  - positivity limiter (Zhang & Shu 2010) per element on every stage
 *    state: with the cell average qbar (weights int l_i), if min rho < delta
 *    q <- qbar + theta1 (q - qbar), theta1 = (rhobar - delta)/(rhobar - min rho);
 *    then if a nodal pressure p_i < delta, q <- qbar + theta2 (q - qbar),
 *    theta2 = min (pbar - delta)/(pbar - p_i), pbar = p(qbar); averages are
 *    kept, an element whose average is not admissible is left as it is. */
typedef struct {
  double s0;     /* indicator threshold (suggested -(1 + 4 log10 p)) */
  double kappa;  /* half-width of the ramp, > 0 (suggested 1) */
  double c_eps;  /* viscosity scale, >= 0 (suggested 0.5) */
  double delta;  /* positivity floor of density and pressure, > 0 (suggested 1e-10) */
} dg_av_params;

/* Indicator and viscosity of q per element (s_out, eps_out: device [E]; s_out
 * may be NULL) and the viscous fluxes G_out: device [3][5][E][Np]
 * (direction-major), which dg_hex_av_rhs also forms.  G is written only in
 * elements with eps > 0 (in the others it is zero and left unwritten). */
dg_status dg_hex_av_viscosity(dg_hex_mesh m, const dg_params* prm, const dg_av_params* av, const double* q,
                              double* s_out, double* eps_out, double* G_out, hipStream_t stream);
/* Euler right-hand side plus the artificial-viscosity term; work: device,
 * at least DG_HEX_AV_RHS_WORK E Np + 2 E doubles (viscous fluxes,
 * indicator, viscosity). */
#define DG_HEX_AV_RHS_WORK 15
dg_status dg_hex_av_rhs(dg_hex_mesh m, const dg_params* prm, const dg_av_params* av, const double* q, double* rhs,
                        double* work, hipStream_t stream);
/* The positivity limiter applied to q in place (asynchronous). */
dg_status dg_hex_limit(dg_hex_mesh m, const dg_params* prm, const dg_av_params* av, double* q, hipStream_t stream);
/* One LSRK(5,4) step with artificial viscosity, each stage state limited;
 * work: at least DG_HEX_SHOCK_STEP_WORK E Np + 2 E doubles. */
#define DG_HEX_SHOCK_STEP_WORK 25
dg_status dg_hex_shock_rk_step(dg_hex_mesh m, const dg_params* prm, const dg_av_params* av, double* q, double* work,
                               double t, double dt, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* DG_HEX_H */
