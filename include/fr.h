/*
 * fr.h -- C ABI of the MI355X flux reconstruction right-hand-side library.
 *
 * The library evaluates the semi-discrete FR right-hand side du/dt of the
 * compressible Euler and Navier-Stokes equations on unstructured quad,
 * triangle and hexahedral meshes (Witherden, Farrington & Vincent, section 2:
 * eqs. ufpts, commsoln, transqu, gradufpts, tnormfluxf, commpflux, tdivflux,
 * negdivconf; physics from section 4 and Appendix B), and advances it with
 * classical RK4.  Operator applications use the matrix form of Appendix A.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every function returns fr_status; nothing throws across the ABI or
 *    aborts.  On failure fr_last_error() holds a message.
 *  - State arrays (u, dudt, lam, ulam) are DEVICE float64 arrays in the
 *    public layout: element blocks concatenated in input order; block b
 *    starts at offset[b] and is indexed [rho][alpha][n] with leading
 *    dimension ld[b] >= nelem (fr_get_layout), i.e. the structure-of-arrays
 *    packing of the paper's implementation section.  Entries with
 *    n >= nelem are padding: they are read but never influence real
 *    entries, and outputs there are written as zero.
 *  - Field order (rho, rho v_x, rho v_y[, rho v_z], E) (eq. eulerflux).
 *  - Solution points: tensor Gauss-Legendre with xi fastest in quads and
 *    hexes; warp-and-blend (alpha = 0) points in triangles, in rows of
 *    increasing eta.  fr_get_solution_points returns their physical
 *    coordinates.
 *  - Calls are stream ordered and asynchronous: they enqueue work on
 *    `hip_stream` (a hipStream_t; NULL = the default stream) and return.
 *    Device-side failures surface at the next synchronising call.
 *  - One context may be used by one host thread at a time.
 */
#ifndef FR_H
#define FR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fr_ctx fr_ctx;

typedef enum {
  FR_OK = 0,
  FR_EINVAL = 1,        /* bad argument (null pointer, bad size, bad enum)   */
  FR_EMESH = 2,         /* det J <= 0, or flux points not paired one-to-one  */
  FR_EUNSUPPORTED = 3,  /* (element type, order) not built into the library  */
  FR_ENOMEM = 4,        /* device or host allocation failed                  */
  FR_EDEVICE = 5,       /* a HIP runtime call failed                         */
  FR_ENONFINITE = 6     /* check_finite found NaN/Inf in the state           */
} fr_status;

typedef enum { FR_QUAD = 0, FR_TRI = 1, FR_HEX = 2 } fr_etype;
typedef enum { FR_EULER = 0, FR_NAVIER_STOKES = 1 } fr_system;
/* Precision of the operator matrix products and the arrays they read and
 * write (flux-point solution, gradients, transformed fluxes).  The state,
 * du/dt, RK registers, metric terms and point-wise arithmetic stay FP64. */
typedef enum { FR_FP64 = 0, FR_FP32 = 1, FR_BF16X3 = 2 } fr_prec;

typedef struct {
  int32_t ndims;          /* 2 or 3                                            */
  int32_t system;         /* fr_system                                         */
  int32_t prec;           /* fr_prec                                           */
  int32_t check_finite;   /* 1: fr_rk_step checks the state, FR_ENONFINITE     */
  double gamma;           /* ratio of specific heats                           */
  double mu;              /* dynamic viscosity (Navier-Stokes)                 */
  double prandtl;         /* Prandtl number (Navier-Stokes)                    */
  double ldg_beta;        /* LDG common-solution bias beta (Navier-Stokes)     */
  double ldg_tau;         /* LDG penalty tau (Navier-Stokes)                   */
  int32_t nproblems;      /* independent problems in the mesh (>= 1)           */
  int32_t autotune;       /* 1: time every GEMM tile plan at set-up, keep the
                             fastest (memoised per shape in the process)       */
} fr_config;

/* Correction functions (section 2, eq. corfn).  DG is the mass-matrix
 * lifting; SD and HU are the members of the VCJH energy-stable family that
 * the super-accuracy test of the validation section compares with DG, built
 * on quads and hexes only (tensor products of the 1-D functions along each
 * face normal). */
typedef enum { FR_CORR_DG = 0, FR_CORR_SD = 1, FR_CORR_HU = 2 } fr_correction;

typedef struct {          /* one element block: one type, order, geometry order */
  int32_t etype;          /* fr_etype                                          */
  int32_t order;          /* solution order p: quad/tri 1..6, hex 1..4         */
  int32_t geom_order;     /* 1 (straight) or 2 (quadratic)                     */
  int32_t correction;     /* fr_correction; SD and HU on triangles give
                             FR_EUNSUPPORTED, other values FR_EINVAL           */
  int64_t nelem;          /* >= 1, and N_V nelem < 2^29 (split larger meshes) */
  const double *nodes;    /* HOST [nelem][nnodes][ndims]; nodes tensor-
                             lexicographic (xi fastest) on {-1,1} or {-1,0,1}
                             for quads/hexes; triangles v0, v1, v2 then the
                             v0v1, v1v2, v2v0 midpoints                        */
  const int32_t *problem; /* HOST [nelem] problem id, or NULL (all problem 0)  */
} fr_block;

typedef struct {          /* one conforming face pair: x_R + shift == x_L       */
  int32_t lblock;
  int32_t lface;          /* quad: 0 eta=-1, 1 xi=+1, 2 eta=+1, 3 xi=-1;
                             tri: 0 v0v1, 1 v1v2, 2 v2v0; hex: 0 zeta=-1,
                             1 eta=-1, 2 xi=+1, 3 eta=+1, 4 xi=-1, 5 zeta=+1   */
  int64_t lelem;
  int32_t rblock;
  int32_t rface;
  int64_t relem;
  double shift[3];        /* periodic translation, zero otherwise             */
} fr_facepair;

/* Boundary conditions (Appendix C), given through ghost states of the
 * boundary element's solution u_L at each boundary flux point. */
typedef enum {
  FR_BC_SUPERSONIC_INFLOW = 0,    /* ghost: the free stream (rho, v, p)        */
  FR_BC_SUBSONIC_OUTFLOW = 1,     /* ghost: rho_L, v_L with the pressure p      */
  FR_BC_NOSLIP_ISOTHERMAL_WALL = 2 /* inviscid ghost: rho_L, 2 v_w - v_L and
                                     energy rho_L (C_p T_w / gamma + |.|^2/2);
                                     LDG ghost: rho_L, v_w, rho_L (C_p T_w /
                                     gamma + |v_w|^2/2); ghost gradient q_L    */
} fr_bctype;

typedef struct {          /* one boundary condition                           */
  int32_t type;           /* fr_bctype                                         */
  int32_t reserved;
  double rho;             /* free-stream density (inflow)                      */
  double v[3];            /* free-stream velocity (inflow)                     */
  double p;               /* free-stream pressure (inflow, outflow)            */
  double cp_tw;           /* C_p T_w (wall)                                    */
  double vw[3];           /* wall velocity (wall)                              */
} fr_bc;

typedef struct {          /* one element face on the domain boundary           */
  int32_t block;
  int32_t face;           /* numbering as in fr_facepair                       */
  int64_t elem;
  int32_t bc;             /* index into the fr_bc array                        */
  int32_t reserved;
} fr_bcface;

/* Build a context: reference operators (Appendix A: M0, M3, M4-M6 M0,
 * M1-M3 M2, M6, block-diagonal M5), per-point metric terms (section 2), the
 * flux-point pair table (each pair visited once, eq. commsoln) and scratch.
 * `blocks`, `pairs` and node arrays are host memory, only read during the
 * call.  fr_setup_mesh: periodic meshes; every flux point must be paired
 * exactly once, else FR_EMESH.  On success *out owns all device memory it
 * allocated. */
fr_status fr_setup_mesh(const fr_config *cfg, int32_t nblocks, const fr_block *blocks,
                        int64_t npairs, const fr_facepair *pairs, void *hip_stream,
                        fr_ctx **out);
/* fr_setup_mesh with boundary faces (Appendix C): every flux point must be
 * paired, or lie on one of the `nbcfaces` boundary faces, exactly once (else
 * FR_EMESH).  At a boundary flux point the common solution is
 * (1/2 - beta) u_L + (1/2 + beta) g_ldg and the common normal flux is the
 * Rusanov flux of (u_L, g_inv) minus n.[(1/2 + beta) f_v(u_L, q_L) +
 * (1/2 - beta) f_v(g_ldg, g_q)] plus tau (u_L - g_ldg), the boundary element
 * being the L side.  `bcs` and `bcfaces` are host memory.  The adjoint calls
 * return FR_EUNSUPPORTED on a context with boundary faces. */
fr_status fr_setup_mesh_bc(const fr_config *cfg, int32_t nblocks, const fr_block *blocks,
                           int64_t npairs, const fr_facepair *pairs, int32_t nbcs,
                           const fr_bc *bcs, int64_t nbcfaces, const fr_bcface *bcfaces,
                           void *hip_stream, fr_ctx **out);

/* Layout of block `block`: its offset into the state array, leading
 * dimension, points per element, fields, and the total state length. */
fr_status fr_get_layout(const fr_ctx *ctx, int32_t block, int64_t *offset, int64_t *ld,
                        int32_t *nupts, int32_t *nvars, int64_t *total_len);

/* Physical solution-point coordinates of block `block` into HOST memory
 * `xyz`, shape [nelem][nupts][ndims]. */
fr_status fr_get_solution_points(const fr_ctx *ctx, int32_t block, double *xyz);

/* Quadrature weights times det J at solution points of block `block` into
 * HOST memory `wj` [nupts][nelem] (integration of solution fields). */
fr_status fr_get_quadrature(const fr_ctx *ctx, int32_t block, double *wj);

/* du/dt = -J^-1 div~ f~ (eq. negdivconf) for the device state u.  dudt may
 * alias u. */
fr_status fr_rhs(fr_ctx *ctx, const double *u, double *dudt, void *hip_stream);

/* nsteps classical RK4 steps in place on u: the classical four-stage
 * Runge-Kutta scheme, one of the time steppers in the functionality table
 * (Table 1) of the paper's implementation section, advancing the
 * semi-discrete system du/dt = R(u) of eq. negdivconf.  dt_dev: DEVICE float64
 * [nproblems], one step size per problem (read on the device, so replays of
 * the captured step graphs pick up new values).  Steps go out in captured
 * graphs of 8 steps while 8 or more remain, then one step per graph; both
 * give the same result bit for bit. */
fr_status fr_rk_step(fr_ctx *ctx, double *u, const double *dt_dev, int32_t nsteps,
                     void *hip_stream);

/* The other time steppers of the paper's functionality table (Table 1 of
 * the implementation section): forward Euler and adaptive DOPRI5.
 *
 * fr_euler_step: nsteps steps u <- u + dt R(u) in place, dt_dev and the
 * captured graphs (8 steps, then one) as for fr_rk_step.
 *
 * fr_dopri5_step: `nattempts` attempts of the Dormand-Prince 5(4) pair in
 * place on u, each problem on its own.  All step-size state is DEVICE
 * float64 memory of [nproblems] entries, read and updated by the kernels
 * (no host synchronisation; attempts replay one captured graph):
 *   t      time of each problem, advanced by accepted steps;
 *   dt     the next step to try; replaced by the controller's proposal;
 *   tend   NULL, or end times: steps are cut to reach them exactly and a
 *          problem at its end time stands still (dt <= 0 also stands still);
 *   counts NULL, or DEVICE int32 [nproblems][2]: accepted and rejected
 *          attempts are added to it.
 * The error of an attempt is the RMS over the problem's degrees of freedom
 * of e_i / (atol + rtol max(|u_i|, |u5_i|)), e = h sum (b_j - bhat_j) k_j;
 * the step is accepted when it is below 1.  The next step is h min(10,
 * 0.9 err^-1/5) after an acceptance (10 when err = 0; at most h when the same
 * step had a rejection) and h max(0.2, 0.9 err^-1/5) after a rejection.  The
 * rejection flag of each problem lives in the context between calls, so a
 * step may span calls.  Each call evaluates R(u) once before its attempts
 * (the first stage), then six right-hand sides per attempt.  atol, rtol > 0
 * and finite, else FR_EINVAL. */
fr_status fr_euler_step(fr_ctx *ctx, double *u, const double *dt_dev, int32_t nsteps,
                        void *hip_stream);
fr_status fr_dopri5_step(fr_ctx *ctx, double *u, double *t, double *dt, const double *tend,
                         int32_t nattempts, double atol, double rtol, int32_t *counts,
                         void *hip_stream);

/* Vector-Jacobian product of the right-hand side: ulam = (dR/du)(u)^T lam.
 * ulam must not alias u or lam. */
fr_status fr_rhs_adjoint(fr_ctx *ctx, const double *u, const double *lam, double *ulam,
                         void *hip_stream);

/* Adjoint of one RK4 step from u_n: lam_n = (d u_{n+1} / d u_n)^T lam_np1.
 * Recomputes the four stages internally.  lam_n may alias lam_np1. */
fr_status fr_rk_step_adjoint(fr_ctx *ctx, const double *u_n, const double *dt_dev,
                             const double *lam_np1, double *lam_n, void *hip_stream);

/* Stashed RK4 step and its adjoint (checkpointed gradients without
 * recomputation).  fr_stash_len gives the size (float64 elements) of one
 * step's stash.  fr_rk_step_stash advances u by one RK4 step like
 * fr_rk_step (not through the graph) and leaves in `stash` (DEVICE, caller
 * owned) the four stage states and their primal intermediates.
 * fr_rk_step_adjoint_stash computes lam_n = (d u_{n+1}/d u_n)^T lam_np1 from
 * that stash with no recomputation; lam_n may alias lam_np1.  FP64 contexts
 * only (FR_EUNSUPPORTED otherwise). */
fr_status fr_stash_len(const fr_ctx *ctx, int64_t *len);
fr_status fr_rk_step_stash(fr_ctx *ctx, double *u, const double *dt_dev, double *stash,
                           void *hip_stream);
fr_status fr_rk_step_adjoint_stash(fr_ctx *ctx, double *stash, const double *dt_dev,
                                   const double *lam_np1, double *lam_n, void *hip_stream);

/* Adjoint of one checkpoint segment of RK4 steps (the checkpointed
 * gradient of the time-stepping scheme of section 2 with the classical RK4
 * scheme of Table 1): replays nsteps steps forward from u_seg0 (DEVICE,
 * read only) while stashing every step into `stash` (DEVICE, caller-owned
 * workspace of nsteps * fr_stash_len float64), then applies the step
 * adjoints from the last step to the first:
 *   lam_seg0 = (d u_{n0+nsteps} / d u_{n0})^T lam_end.
 * lam_seg0 may alias lam_end; stash must overlap neither, nor u_seg0.  The
 * whole segment runs as one HIP graph, captured on the first call with a
 * given (u_seg0, dt_dev, nsteps, lam_end, lam_seg0, stash) and replayed on
 * later calls with the same arguments (the context keeps the last four);
 * callers that keep those buffers at fixed addresses pay the capture once.
 * The stash contents are overwritten.  nsteps = 0 copies lam_end to
 * lam_seg0.  FP64 contexts without boundary conditions
 * (FR_EUNSUPPORTED otherwise); FR_EINVAL for null pointers or nsteps < 0. */
fr_status fr_rk_segment_adjoint(fr_ctx *ctx, const double *u_seg0, const double *dt_dev,
                                int32_t nsteps, const double *lam_end, double *lam_seg0,
                                double *stash, void *hip_stream);

/* Integrals of the state by quadrature at the solution points (paper's
 * validation section: sums of W J times the integrand).  kind must be 0:
 * out (DEVICE float64) [nproblems][nvars + 1] receives, per problem, the
 * integral of every conserved field followed by the kinetic energy
 * |rho v|^2 / (2 rho).  Summation order is fixed (bitwise reproducible). */
fr_status fr_integrate(fr_ctx *ctx, const double *u, int32_t kind, double *out,
                       void *hip_stream);

/* fr_integrate for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops or harnesses that forbid hipMalloc).
 * Same arguments, kernels, summation order and result as fr_integrate
 * (bitwise), but the element and slice partials live in a fixed scratch
 * array inside the library, one copy per GPU, held until the process ends:
 * FR_INTEGRAL_SCRATCH_DOUBLES doubles (32 MiB).  Its address on a device is
 * resolved once, when the first context is set up there.  The call allocates
 * nothing and needs no clearing (every partial it reads it writes first).
 * A mesh whose partials need more than the fixed scratch holds
 * (nchunk x elements x (nvars + 1) plus the slice partials; about 800,000
 * elements of a 3-D mesh) gets FR_EINVAL with a message naming both sizes.
 * Every call on one GPU shares that GPU's scratch: calls that overlap in
 * time on one GPU (other streams, other threads) race and must be ordered
 * by the caller. */
#define FR_INTEGRAL_SCRATCH_DOUBLES 4194304
fr_status fr_integrate_noalloc(fr_ctx *ctx, const double *u, int32_t kind, double *out,
                               void *hip_stream);

/* Host-only diagnostics (no device use; callable without a GPU).
 * fr_reference_operator copies one reference-element array of (etype, p,
 * fr_correction) into HOST memory `out` (capacity `cap` doubles) and stores its shape in
 * rows/cols.  which: 0 M0 (Nf x Nu), 1 M3 (Nu x Nf), 2 M4 - M6 M0
 * (D Nu x Nu), 3 M6 (D Nu x Nf), 4 M1 - M3 M2 (Nu x D Nu), 5 solution
 * points (Nu x D), 6 flux points (Nf x D), 7 reference normals (Nf x D),
 * 8 quadrature weights W (Nu x 1), 9 face weights omega (Nf x 1), 10 M4
 * (D Nu x Nu), 11 M1 (Nu x D Nu).  Out-of-range `which` or too small `cap`
 * gives FR_EINVAL; an unsupported order FR_EUNSUPPORTED.
 * fr_check_mesh runs the host part of fr_setup_mesh (metric terms and flux
 * point pairing) and returns its status; npoint_pairs receives the number of
 * flux-point pairs. */
fr_status fr_reference_operator(int32_t etype, int32_t order, int32_t correction, int32_t which,
                                double *out, int64_t cap, int32_t *rows, int32_t *cols);
fr_status fr_check_mesh(const fr_config *cfg, int32_t nblocks, const fr_block *blocks,
                        int64_t npairs, const fr_facepair *pairs, int64_t *npoint_pairs);

/* Device diagnostics (test support).
 * fr_debug_stage runs the right-hand-side chain of an FP64 context up to
 * step `stage` (1: U^f = M0 U, 2: common solution C^f, 3: Q~, 4: Q = J^-T Q~,
 * 5: Q^f, 6: transformed flux F~, 7: D~ = common normal flux) and copies
 * that internal array (layout [row][alpha][ld] per block, blocks
 * concatenated) into the DEVICE buffer `out` of fr_debug_scratch_len
 * doubles.  fr_debug_gemm computes C = A [B1; B2] with the library's matrix
 * core kernel: A HOST row-major M x (K1 + K2); B1 (K1 rows), B2 (K2 rows)
 * DEVICE float64 with row stride ldb >= N; C DEVICE (float64 for FP64, float32
 * for FP32) M x N, row stride N; N a multiple of 16.  (mbw, nc, wm) forces a
 * matrix-core tile plan; mbw = 0 with nc > 0 and wm = 0 forces the
 * sparse-row kernel, one column per thread, with nc operator rows per
 * workgroup (FR_EINVAL if A is not sparse: at
 * least half of its entries must be zero, or below 1e-13 of their row's
 * largest magnitude); mbw = nc = 0: the default plan.  Synchronous. */
fr_status fr_debug_stage(fr_ctx *ctx, const double *u, int32_t stage, double *out,
                         void *hip_stream);
fr_status fr_debug_scratch_len(const fr_ctx *ctx, int32_t stage, int64_t *len);
/* Benchmark hook: prepares the inputs of right-hand-side step `step` (as
 * numbered for fr_debug_stage, plus 8: the final product with du/dt) for
 * state u, then launches that step's kernels nrep times on hip_stream (step
 * 7 works in place, so its repeats read the previous repeat's output; the
 * values are meaningless, the work is the same).  The output of step 8 goes
 * to internal scratch.  Step 9: step 8 with the RK4 register update of a
 * middle stage, as the captured step graph runs it (reads u and the
 * accumulator, writes the accumulator and the next stage; internal
 * registers, dt = 0). */
fr_status fr_bench_step(fr_ctx *ctx, const double *u, int32_t step, int32_t nrep,
                        void *hip_stream);
fr_status fr_debug_gemm(int32_t prec, int32_t M, int32_t K1, int32_t K2, const double *A,
                        const void *B1, const void *B2, int64_t ldb, void *C, int64_t N,
                        int32_t mbw, int32_t nc, int32_t wm, void *hip_stream);

/* Performance diagnostics.
 * fr_measure_ceiling: kind 0 = HBM triad bandwidth (GB/s, 3 x 2 GiB arrays),
 * 1 = FP64 matrix-core rate, 2 = FP32 matrix-core rate (TFLOP/s,
 * register-resident v_mfma loops).  Synchronous.
 * fr_bench_gemm: average time of one launch of the operator GEMM kernel for
 * an M x (K1 + K2) operator on N columns (batch copies of panel 1) with tile
 * plan (mbw, nc, wm) (mbw = 0: default plan); operands are internal.
 * fr_get_gemm_plan: the tile plan a context uses for right-hand-side step
 * 1, 3, 5 or 8 of `block`.  mbw = 0: the sparse-row kernel with nc
 * operator rows per workgroup and wm a set of flags: bit 0 (step 3 only)
 * the gradient transform of step 4 fused into its epilogue, so that step 4
 * launches nothing; bit 1 every field of an element computed by one thread;
 * bit 2 the LDS-staged kernel (64 columns and all rows per workgroup, B
 * streamed through LDS; nc is then unused and reported as 64); bit 3 (step
 * 3, with bits 0 and 1) the transformed flux of step 6 computed in the same
 * epilogue, so that step 6 launches nothing. */
fr_status fr_measure_ceiling(int32_t kind, double *value, void *hip_stream);
fr_status fr_bench_gemm(int32_t prec, int32_t M, int32_t K1, int32_t K2, int64_t N,
                        int32_t mbw, int32_t nc, int32_t wm, int32_t batch, int32_t nrep,
                        float *ms_per_launch, void *hip_stream);
fr_status fr_get_gemm_plan(const fr_ctx *ctx, int32_t block, int32_t step, int32_t *mbw,
                           int32_t *nc, int32_t *wm);
/* fr_debug_set_plan forces the plan of right-hand-side step 1, 3, 5 or 8 of
 * `block`, or (FP64 contexts) of the adjoint's M0^T product (step 13), which
 * with a sparse-row plan also applies the reverse gradient transform, or of
 * its (M1 - M3 M2)^T product (step 14), where flags 2 | 16 apply the reverse
 * of the transformed flux in the epilogue (test support: drives every
 * kernel variant through the full chain): mbw > 0 a
 * matrix-core plan (mbw, nc, wm) as for fr_debug_gemm;
 * mbw = 0 the sparse-row kernel with nc rows per workgroup and the flags
 * wm of fr_get_gemm_plan (fusion with bit 1 needs an operator of at most 16
 * non-zeros per row; bit 2 excludes bit 1 and needs at most 160 rows, or
 * 64 points when fused).  FR_EINVAL for an invalid plan
 * or an operator without a sparse form.  Drops the captured RK4 graph.
 * Synchronous on hip_stream. */
fr_status fr_debug_set_plan(fr_ctx *ctx, int32_t block, int32_t step, int32_t mbw, int32_t nc,
                            int32_t wm, void *hip_stream);

/* Multi-block launches (test and report support).  On a mesh of several
 * element blocks the set-up times, for steps 1 (U^f = M0 U), 5 (Q^f), 8 (the
 * divergence with its epilogue) and 6 (transformed flux), one launch per
 * kernel family over every block against a launch per block, and keeps the
 * faster.  fr_debug_multi reports (state: bit 0 sparse-row launch over
 * several blocks, bit 1 matrix-core launch over several blocks, bit 2 for
 * step 6 the one-launch transformed flux) and, with mode >= 0, sets it: 0 a
 * launch per block, 1 one launch per family with one field per thread (and
 * one column strip per wavefront), 2 with all fields per thread (two
 * strips).  A plan forced with fr_debug_set_plan turns that step's
 * multi-block launches off.  FP64 and FP32 contexts; BF16x3 launches per
 * block.  Steps other than 1, 5, 6, 8 give FR_EINVAL. */
fr_status fr_debug_multi(fr_ctx *ctx, int32_t step, int32_t mode, int32_t *state,
                         void *hip_stream);

/* Gradient of an integral of fr_integrate with respect to the state: kind 1
 * (kinetic energy, summed over problems) -> grad (DEVICE, state layout),
 * W J (-|v|^2 / 2, v, 0) at each solution point. */
fr_status fr_integrate_grad(fr_ctx *ctx, const double *u, int32_t kind, double *grad,
                            void *hip_stream);

/* Message of the last failure on ctx (ctx NULL: last failed setup on this
 * thread).  Never NULL. */
const char *fr_last_error(const fr_ctx *ctx);

/* Release every resource owned by ctx (after synchronising its stream). */
void fr_destroy(fr_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* FR_H */
