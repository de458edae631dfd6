/*
 * cgp.h -- C ABI of the MI355X (gfx950) coarse-grid incremental
 * pressure-projection (CGP) library.
 *
 * The method (Kashefi, "A coarse-grid incremental pressure-projection method
 * for accelerating low Reynolds number incompressible flow simulations"):
 * each time step solves a fine-mesh momentum problem for the intermediate
 * velocity (Eq. 21), restricts it to a mesh coarsened by k levels of uniform
 * 4:1 refinement (Eq. 22), solves the pressure-increment Poisson problem there
 * (Eq. 23), prolongs the increment back (Eq. 24) and corrects velocity and
 * pressure on the fine mesh (Eqs. 25-26, Sect. 2.3).
 *
 * Conventions shared by every entry point
 *  - Return value: CGP_OK (0), CGP_NOT_CONVERGED (1, outputs written and stats
 *    valid) or a negative error code.  cgp_last_error() returns a
 *    thread-local message describing the last failure.  Nothing throws across
 *    the ABI and nothing calls exit().
 *  - Host pointers are read during the call only.  Device pointers are owned
 *    by the caller and must stay valid until the work queued on `stream` has
 *    finished.  `stream` is a hipStream_t passed as void* (NULL = the null
 *    stream).  Device work is queued on `stream`; a call returns before it
 *    finishes unless stated otherwise.
 *  - The library allocates no device or pinned host memory.  cgp_query()
 *    reports the size of the device workspace and of the small page-locked
 *    host buffer (convergence flags the kernels mirror for the host to poll)
 *    that the caller provides to cgp_assemble().
 *  - Node numbering of the fine mesh (the only numbering seen at the ABI):
 *    refinement level by level appends the midpoint of every edge in
 *    first-encounter order over (triangle, local edge (0,1), (1,2), (2,0));
 *    triangle (a,b,c) with midpoints m_ab, m_bc, m_ca has children
 *    (a,m_ab,m_ca), (m_ab,b,m_bc), (m_ca,m_bc,c), (m_ab,m_bc,m_ca) in that
 *    order, and a boundary edge (p,q) splits into (p,m), (m,q) with the
 *    parent's tag.  The finest level is then numbered: the coarse nodes keep
 *    0..N_c-1, and the new nodes follow, stably sorted by the coarse triangle
 *    that is the ancestor of the triangle that first created them (the nodes
 *    of one coarse triangle are contiguous).  Fine triangles keep their
 *    order: those of coarse triangle T are T*4^k .. (T+1)*4^k - 1.
 *  - Field layout: velocities are structure-of-arrays float64 [2][N_f]
 *    (u then v); scalars float64 [N]; all arrays dense and contiguous.
 */
#ifndef CGP_H
#define CGP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define CGP_OK 0
#define CGP_NOT_CONVERGED 1
#define CGP_ERR_INVALID (-1)   /* bad argument, size or pointer            */
#define CGP_ERR_MESH (-2)      /* clockwise/degenerate/non-conforming mesh */
#define CGP_ERR_HIP (-3)       /* a HIP runtime call failed                */
#define CGP_ERR_NAN (-4)       /* a solver produced NaN/Inf                */
#define CGP_ERR_WORKSPACE (-5) /* workspace missing, too small, misaligned */

/* boundary-edge tags (problem statement, Sect. 2.1, Eqs. 3-4) */
#define CGP_DIRICHLET 1 /* velocity prescribed (Eq. 10); grad(phi).n = 0 (Eq. 13) */
#define CGP_NATURAL 2   /* traction boundary (Eqs. 4, 11): -p n + nu grad(u) n = t_N,
                           with t_N given per step (t_nat below) or 0 when
                           none is given; phi = 0 (Eq. 14)                 */

/* coarse-solve precision */
#define CGP_FP64 0  /* Jacobi-PCG in FP64 throughout */
#define CGP_MIXED 1 /* FP64 iterative refinement around FP32-inner Jacobi-PCG */

/* coarse-solve preconditioner (the paper preconditions its Krylov solves
 * with ILU(0), Sect. 2.3; the choice of coarse solver is open) */
#define CGP_PRECOND_JACOBI 0 /* diagonal: single-reduction PCG, FP64 or mixed   */
#define CGP_PRECOND_NDCHOL 1 /* nested-dissection Cholesky factor of K_c: FP64
                                PCG, or with CGP_MIXED FP64 iterative refinement
                                whose corrections are FP32 factor solves        */
#define CGP_PRECOND_JACOBI_S4 2 /* diagonal, s-step form (FP64): the iterates of
                                  Jacobi-PCG, four iterations per launch from
                                  one Gram-matrix reduction (Chebyshev basis of
                                  the scaled operator); every iteration keeps
                                  the ||b - K phi|| stopping test             */

/* projection scheme */
#define CGP_SCHEME_INCREMENTAL 0    /* the method: Eqs. 21-26 (standard or rotational) */
#define CGP_SCHEME_NONINCREMENTAL 1 /* the non-incremental CGP form the paper compares
                                       with (Sect. 2.3): no pressure in the momentum
                                       equation, Eq. 23 solved for the pressure itself,
                                       P^{n+1} = Phi_f; chi must be 0 */

/* reading of the coarse divergence in Eq. 23 (Sect. 2.2) */
#define CGP_RESTRICT_GALERKIN 0 /* coarse shape functions against the fine velocity */
#define CGP_RESTRICT_INJECT 1   /* inject U~ at the coarse nodes (Eq. 22), then D_c */

/* Coarse (Poisson) mesh; the fine mesh is `levels` uniform refinements of it.
 * Host arrays.  Triangles counter-clockwise with positive area; every
 * boundary edge must be an edge of exactly one triangle. */
typedef struct cgp_mesh {
  int32_t n_nodes;
  int32_t n_tris;
  int32_t n_bedges;
  const double* xy;     /* [2*n_nodes] interleaved (x, y)        */
  const int32_t* tri;   /* [3*n_tris]                            */
  const int32_t* bedge; /* [2*n_bedges] node pairs               */
  const int32_t* btag;  /* [n_bedges] CGP_DIRICHLET / CGP_NATURAL */
} cgp_mesh;

/* The problem statement of Sect. 2.1 (dimensionless; nu = 1/Re) plus the
 * coarsening level k of Sect. 2.2 and the solver settings. */
#define CGP_MASS_CONSISTENT 0
#define CGP_MASS_LUMPED_P 1
#define CGP_MASS_LUMPED 2
#define CGP_MASS_CONSISTENT_MIXED 3

typedef struct cgp_problem {
  cgp_mesh coarse;
  int32_t levels;        /* k in 0..3                                        */
  int32_t chi;           /* 0 standard, 1 rotational form (Eq. 16)           */
  int32_t precision;     /* CGP_FP64 or CGP_MIXED                            */
  int32_t restrict_mode; /* CGP_RESTRICT_GALERKIN or CGP_RESTRICT_INJECT     */
  double dt;             /* time step                                        */
  double nu;             /* kinematic viscosity 1/Re                         */
  double pcg_tol;        /* coarse solve: ||b - K phi||_2 <= pcg_tol ||b||_2  */
  double inner_tol;      /* mixed: floor of the FP32 inner relative tolerance
                            (each inner solve targets max(inner_tol,
                            0.3 pcg_tol ||b|| / ||r_outer||))                 */
  double mom_tol;        /* momentum BiCGSTAB relative tolerance             */
  double mass_tol;       /* consistent mass solves: target of the Chebyshev
                            iteration (sets its fixed step count)            */
  int32_t max_iter;      /* coarse PCG iteration cap (all inner iterations)  */
  int32_t mom_max_iter;  /* momentum iteration cap                           */
  int32_t mass_max_iter; /* mass-solve iteration cap                         */
  int32_t max_outer;     /* mixed: refinement-step cap                       */
  int32_t mass_mode;     /* CGP_MASS_CONSISTENT (Eqs. 25, 26), CGP_MASS_LUMPED_P
                            (rotational pressure update with the lumped mass
                            matrix, Eq. 27), CGP_MASS_LUMPED (Eq. 27 and the
                            velocity correction with the lumped mass matrix;
                            no mass solves) or CGP_MASS_CONSISTENT_MIXED (the
                            consistent solves as FP64 iterative refinement:
                            two Chebyshev solves with float-stored iterates,
                            each of the step count for sqrt(mass_tol) plus
                            one, the second on the FP64 residual of the
                            first; the solution is their FP64 sum)          */
  int32_t coarse_precond; /* CGP_PRECOND_JACOBI, CGP_PRECOND_JACOBI_S4 (the same
                            solver in s-step form; requires precision =
                            CGP_FP64; cgp_create fails with CGP_ERR_INVALID
                            if a coarse node's depth-4 graph neighbourhood
                            exceeds 1024 nodes), or CGP_PRECOND_NDCHOL: PCG in
                            FP64 preconditioned by the exact Cholesky factor
                            of K_c (phi = 0 nodes removed; without natural
                            nodes the last coarse node N_c - 1 is pinned, as
                            K_c is singular), computed once on the host in
                            cgp_assemble; with precision = CGP_MIXED the
                            factor is stored in FP32 and the solve is FP64
                            iterative refinement around FP32 factor solves
                            (FP32 storage and accumulation; the residual,
                            its norm and the iterate in FP64)                */
  int32_t scheme;         /* CGP_SCHEME_INCREMENTAL or CGP_SCHEME_NONINCREMENTAL */
} cgp_problem;

typedef struct cgp_sizes {
  int64_t n_fine, n_coarse;          /* nodes                                 */
  int64_t n_fine_tris, n_coarse_tris;
  int64_t nnz_fine, nnz_coarse;      /* CSR nonzeros of the P1 node graphs    */
  int64_t n_dirichlet;               /* fine velocity-Dirichlet nodes         */
  int64_t n_natural_coarse;          /* coarse phi = 0 nodes                  */
  size_t workspace_bytes;            /* device workspace for cgp_assemble     */
  size_t host_bytes;                 /* page-locked host buffer for cgp_assemble */
} cgp_sizes;

/* One linear solve.  iters counts Krylov iterations (inner iterations summed
 * on the mixed path); rel_res is the FP64 relative residual the stopping test
 * last saw (recursive for plain PCG/BiCGSTAB, true for mixed refinement). */
typedef struct cgp_solve_stats {
  int32_t iters;
  int32_t outer_iters;
  int32_t converged;
  int32_t pad_;
  double rel_res;
} cgp_solve_stats;

typedef struct cgp_step_stats {
  cgp_solve_stats momentum[2]; /* u, v                          */
  cgp_solve_stats poisson;     /* coarse pressure increment     */
  cgp_solve_stats mass[2];     /* velocity correction u, v      */
  cgp_solve_stats prot;        /* rotational pressure mass solve */
  int32_t guess_net;           /* 1: the learned guess was used  */
  int32_t pad_;
} cgp_step_stats;

/* Time-stepping state, device pointers owned by the caller.  The step writes
 * U^{n+1} into the buffer that held U^{n-1} and swaps the two pointers, so on
 * return u_prev = U^n and u = U^{n+1}; p is updated in place; phi_hist[0..3]
 * are rotated so that phi_hist[0] holds the new coarse increment. */
typedef struct cgp_state {
  double* u_prev;      /* [2][N_f] U^{n-1}                          */
  double* u;           /* [2][N_f] U^n                              */
  double* p;           /* [N_f]    P^n                              */
  double* phi_hist[4]; /* [N_c] each: coarse increments, newest first */
  int64_t step;
} cgp_state;

typedef struct cgp_ctx cgp_ctx;

/* Host-only set-up: validates the coarse mesh (index range, positive area,
 * conformity, boundary edges), refines it `levels` times and builds every
 * index structure (CSR graphs, edge-side lists, prolongation codes).  No
 * device memory is touched.  *out receives a context to be released with
 * cgp_destroy().  Errors: CGP_ERR_INVALID, CGP_ERR_MESH. */
int cgp_create(const cgp_problem* problem, cgp_ctx** out);

/* Sizes of the refined problem and of the device workspace. */
int cgp_query(const cgp_ctx* ctx, cgp_sizes* out);

/* Fine-mesh node coordinates, host [2*N_f] interleaved (x, y). */
int cgp_fine_nodes(const cgp_ctx* ctx, double* xy_host);

/* Sorted fine velocity-Dirichlet nodes, host [n_dirichlet].  Every node on a
 * CGP_DIRICHLET edge is one (walls win at junctions with the outflow).  The
 * u_dir arrays passed below follow this order. */
int cgp_dirichlet_nodes(const cgp_ctx* ctx, int32_t* nodes_host);

/* Device set-up: carves `workspace` (device, >= workspace_bytes, 256-byte
 * aligned, caller-owned for the life of the context), uploads the index
 * structures and assembles the constant operators (fine mass matrix; coarse
 * stiffness, divergence, lumped masses; Jacobi diagonals).  `host` is
 * page-locked host memory that device kernels can write (hipHostMalloc, or
 * a pinned allocation of the caller's framework), >= host_bytes, 64-byte
 * aligned, caller-owned for the life of the context and not touched by the
 * caller meanwhile: the solver kernels mirror their stopping flags there and
 * the host reads them after an event.  Synchronises `stream` before
 * returning.  Errors: CGP_ERR_WORKSPACE, CGP_ERR_HIP. */
int cgp_assemble(cgp_ctx* ctx, void* workspace, size_t bytes, void* host, size_t host_bytes,
                 void* stream);

/* Step 1 (Eq. 21): solves
 *   (3/2 M + dt N(w) + dt nu K) U~ = -dt G P + dt M F + dt B T + 2 M U - 1/2 M U_prev,
 *   w = 2 U - U_prev, with U~ = u_dir at the Dirichlet nodes (Eq. 10),
 * by right-Jacobi-preconditioned BiCGSTAB from U~ = w (u_dir at the
 * Dirichlet nodes), stopping when
 * ||r|| <= mom_tol ||rhs||.  B T is the traction term of Eq. 11 (Eqs. 4, 8):
 * B the P1 boundary mass matrix of the CGP_NATURAL edges, T the nodal
 * traction t_N(t^{n+1}); with G = -D^T the weak form's natural condition is
 * then -P n + nu grad(U~) n = t_N.  u_prev, u, u_tilde: device [2][N_f]; p device
 * [N_f] (not read, and may be NULL, with CGP_SCHEME_NONINCREMENTAL, whose
 * momentum equation has no pressure term); u_dir device [2][n_dirichlet]; f device [2][N_f] or NULL (no
 * forcing); t_nat device [2][N_f] (read at the nodes of natural edges only)
 * or NULL (traction free; CGP_ERR_INVALID if given without a natural edge).
 * u_tilde must not alias the inputs.  stats may be NULL; when
 * given, the call synchronises `stream` to fill it. */
int cgp_momentum(cgp_ctx* ctx, const double* u_prev, const double* u, const double* p,
                 const double* u_dir, const double* f, const double* t_nat, double* u_tilde,
                 cgp_solve_stats stats[2], void* stream);

/* Steps 2-3, right-hand side (Eqs. 22-23): b_c = -(3/(2 dt)) Dbar U~ with
 * Dbar the coarse divergence selected by restrict_mode; zero at the coarse
 * phi = 0 nodes (Eq. 14); projected onto zero mean when no boundary is
 * natural.  Evaluated in FP64 on both precision paths (a divergence of a
 * nearly solenoidal field is a sum of nearly cancelling terms).  u_tilde
 * device [2][N_f], b_c device [N_c]. */
int cgp_restrict(cgp_ctx* ctx, const double* u_tilde, double* b_c, void* stream);

/* Step 3 (Eq. 23): solves K_c phi_c = b_c (K_c the coarse stiffness matrix,
 * phi = 0 rows/columns removed) from the guess held in phi_c, stopping when
 * ||b - K phi|| <= pcg_tol ||b||; CGP_FP64 runs Jacobi-PCG in FP64,
 * CGP_MIXED runs FP64 refinement steps around FP32 Jacobi-PCG (FP64 dot
 * products and norms); CGP_PRECOND_JACOBI_S4 runs FP64 Jacobi-PCG in s-step
 * form (same iterates up to rounding, same test after every iteration);
 * CGP_PRECOND_NDCHOL runs FP64 PCG whose
 * preconditioner is the factor (one iteration reaches rounding level; the
 * FP64 residual is tested before the first and after every iteration), or,
 * with CGP_MIXED, FP64 refinement steps x += F32^-1 (b - K x), F32 the
 * factor in FP32 (each removes all but about kappa(K_c) eps_32 of the error;
 * the FP64 residual is tested before every correction; stats->iters and
 * outer_iters count the corrections, capped by max_outer).  For the pure Neumann problem the lumped-mass mean of
 * the result is removed.  b_c, phi_c device [N_c].  stats may be NULL (then
 * no synchronisation beyond the convergence polling). */
int cgp_pcg_solve(cgp_ctx* ctx, const double* b_c, double* phi_c, cgp_solve_stats* stats,
                  void* stream);

/* cgp_pcg_solve for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid allocation): the
 * same FP64 Jacobi-PCG, iterates and stopping test, but its Krylov vectors,
 * partial sums and solver scalars live in a file-scope device array of the
 * library (one per GPU, about 7.5 MB, held until the process ends) instead
 * of the context's workspace.  The call allocates nothing, host or device.
 * Requires coarse_precond CGP_PRECOND_JACOBI and precision CGP_FP64
 * (CGP_ERR_INVALID otherwise) and N_c <= 131072 (CGP_ERR_WORKSPACE
 * otherwise).  Every context on a GPU shares that GPU's array and it keeps
 * the last call's contents: calls that overlap on one GPU (two streams, or
 * two host threads) race and must be serialised by the caller.  Arguments,
 * results and status as cgp_pcg_solve. */
int cgp_pcg_solve_noalloc(cgp_ctx* ctx, const double* b_c, double* phi_c,
                          cgp_solve_stats* stats, void* stream);

/* Step 4 (Eq. 24): phi_f = P phi_c, linear interpolation applied k times
 * (each fine node is the coarse P1 function evaluated there; dyadic weights).
 * FP64 on both precision paths: the velocity correction differentiates
 * phi_f, which would amplify FP32 rounding of a large increment.
 * phi_c device [N_c], phi_f device [N_f]. */
int cgp_prolong(cgp_ctx* ctx, const double* phi_c, double* phi_f, void* stream);

/* Steps 5-6 (Eqs. 25-26, Sect. 2.3): M dU = -(2/3) dt G phi_f on the
 * non-Dirichlet nodes (consistent mass), u_out = u_tilde + dU; p_out =
 * p_in + phi_f for chi = 0; for chi = 1 additionally M dp = -nu D u_tilde and
 * p_out = p_in + phi_f + dp.  The mass solves run together as Chebyshev
 * iteration on [1/2, 2] (the spectrum of the Jacobi-scaled P1 mass matrix),
 * with the iteration count fixed by mass_tol (27 for 1e-12); stats report
 * that count and its a-priori error bound.  With CGP_MASS_CONSISTENT_MIXED
 * stats report both solves' steps (iters, 2 x 15 for 1e-12), outer_iters 2,
 * and as rel_res the square of the inner bound plus 8 float ulps (an
 * estimate: the float storage is not bounded a priori).  With CGP_SCHEME_NONINCREMENTAL
 * p_out = phi_f (p_in not read, may be NULL).  p_out may alias p_in.
 * u_tilde, u_out device [2][N_f]; phi_f, p_in, p_out device [N_f].  stats:
 * [3] (u, v, rotational) or NULL. */
int cgp_correct(cgp_ctx* ctx, const double* u_tilde, const double* phi_f, const double* p_in,
                double* u_out, double* p_out, cgp_solve_stats stats[3], void* stream);

/* One whole CGP step (Eqs. 21-26): momentum, restriction, coarse solve from
 * the guess phi_hist[0] (or `guess` when not NULL), prolongation,
 * correction; then rotates the state as described at cgp_state.  u_dir
 * device [2][n_dirichlet] at t^{n+1}; f device [2][N_f] or NULL; t_nat
 * device [2][N_f] at t^{n+1} or NULL (as in cgp_momentum); guess
 * device [N_c] or NULL.  stats may be NULL; when given the call
 * synchronises `stream` to fill it. */
int cgp_project_step(cgp_ctx* ctx, cgp_state* state, const double* u_dir, const double* f,
                     const double* t_nat, const double* guess, cgp_step_stats* stats,
                     void* stream);

/* ---- Learned initial guess for the coarse solve ------------------------
 * Not part of the paper's method: an accelerator of step 3.  A 3-round
 * message-passing network (hidden width 32) on the coarse node graph maps
 * the coarse right-hand side b and the last four solutions phi^n ... phi^{n-3}
 * (newest first) to a predicted solution: it refines the FP64 quadratic
 * extrapolation q = 3 phi^n - 3 phi^{n-1} + phi^{n-2} in units of
 * s = rms(e), e = phi^n - 3 phi^{n-1} + 3 phi^{n-2} - phi^{n-3} (the error
 * that extrapolation made one step earlier; floored at 1e-12 rms(phi^n),
 * else rms(b) / hbar^2 with hbar the mean coarse edge length).  Node inputs:
 * b / rms(b), (b - K q) / s, e / s, and the first and second differences of
 * the history over their own rms; output q + s y.  Its dense layers run on
 * BF16 MFMA with FP32 accumulation.  The coarse solve then starts from the prediction only if
 * its FP64 residual ||b - K x0|| is not larger than that of the previous
 * increment, and always runs to pcg_tol, so the result never depends on the
 * network beyond the solver tolerance.
 * Parameters: CGP_NET_PARAMS float32 values, device, caller-owned, in the
 * order W_e [32][5], c_e [32], then per round A [32][32], B [32][32],
 * C [32][3], d [32], U [32][64], v [32], then w [32], c [1] (row-major,
 * output x input).  `hist` is a host array of 4 device pointers [N_c]. */
#define CGP_NET_PARAMS 12993

/* Seeded fan-in uniform initialisation of a host parameter vector. */
int cgp_net_init(float* theta_host, uint64_t seed);

/* guess [N_c] (device) = the network's predicted solution. */
int cgp_net_guess(cgp_ctx* ctx, const float* theta, const double* b_c,
                  const double* const* hist, double* guess, void* stream);

/* Gradient (device float [CGP_NET_PARAMS], may be NULL) and loss (device
 * float, may be NULL) of the mean squared error between the prediction and
 * target (the solved phi^{n+1}), as y against t = (target - q) / s, divided
 * by max(1, mean t^2) so that samples whose history is dominated by solver
 * noise carry bounded weight. */
int cgp_net_grad(cgp_ctx* ctx, const float* theta, const double* b_c,
                 const double* const* hist, const double* target, float* grad, float* loss,
                 void* stream);

/* One Adam step (beta 0.9, 0.999, eps 1e-8; step counts from 1) on theta
 * with moments m, v (device float [CGP_NET_PARAMS], caller-owned). */
int cgp_net_train_step(cgp_ctx* ctx, float* theta, float* m, float* v, int32_t step, float lr,
                       const double* b_c, const double* const* hist, const double* target,
                       float* loss, void* stream);

/* The network-free candidate the network refines: q = 3 hist[0] -
 * 3 hist[1] + hist[2] (quadratic extrapolation of the last three coarse
 * increments), 0 at the phi = 0 nodes.  hist: host array of 3 (or 4) device
 * pointers [N_c]; q device [N_c], may not alias them. */
int cgp_extrapolate(cgp_ctx* ctx, const double* const* hist, double* q, void* stream);

/* Copies whichever of cand and prev (device [N_c]) has the smaller FP64
 * residual against the coarse system (cand on ties) into out; *chose
 * (device int32, may be NULL) receives 0 for cand, 1 for prev. */
int cgp_guess_guard(cgp_ctx* ctx, const double* b_c, const double* cand, const double* prev,
                    double* out, int32_t* chose, void* stream);

/* cgp_project_step with the guarded learned guess for the coarse solve;
 * stats->guess_net reports whether the network's candidate was used. */
int cgp_project_step_net(cgp_ctx* ctx, cgp_state* state, const double* u_dir, const double* f,
                         const double* t_nat, const float* theta, cgp_step_stats* stats,
                         void* stream);

/* Device buffers of the last step's intermediates (read-only views into the
 * workspace, valid until the next call on ctx): U~ [2][N_f], b_c [N_c],
 * phi_f [N_f].  Any argument may be NULL. */
int cgp_intermediates(cgp_ctx* ctx, const double** u_tilde, const double** b_c,
                      const double** phi_f);

/* Measurement hook.  While enabled, every launch of the selected kernel on
 * this context is bracketed by a pair of HIP events recorded on the stream
 * the kernel runs on.  kernel_id: 0 off, CGP_K_MASS_SPMV (one Chebyshev step
 * of the fused mass-matrix solves -- velocity correction and, for chi = 1, the
 * rotational pressure update -- after the first, over all lattice nodes or,
 * with lattice size 8, over the coarse-edge and vertex nodes),
 * CGP_K_MASS_PAIR (lattice size 8: two Chebyshev steps on the interior
 * nodes of the coarse triangles), CGP_K_MOM_SPMV (momentum BiCGSTAB product
 * v = A p^, 2 right-hand sides), CGP_K_COARSE_SPMV (coarse PCG product
 * kernel), CGP_K_MOM_ASSEMBLE (momentum matrix and right-hand side).
 * Enabling resets the accumulated time.  cgp_timing_read synchronises the
 * recorded events and returns the summed kernel time (ms) and the number of
 * launches. */
#define CGP_K_MASS_SPMV 1
#define CGP_K_MOM_SPMV 2
#define CGP_K_COARSE_SPMV 3
#define CGP_K_MOM_ASSEMBLE 4
#define CGP_K_MASS_PAIR 5
int cgp_timing_enable(cgp_ctx* ctx, int kernel_id);
int cgp_timing_read(cgp_ctx* ctx, double* total_ms, int64_t* launches);

/* ---- Nested-dissection factor of the coarse matrix ---------------------
 * Structure of the factor used by CGP_PRECOND_NDCHOL: unknowns factored,
 * supernodes (leaves of at most 32 nodes and separators), tree levels (one
 * forward and one backward launch each), the widest front, and the stored
 * factor entries (G = [L11^-1 ; L21 L11^-1] per supernode; the workspace
 * holds it twice, as G and G^T). */
typedef struct cgp_ndchol_info {
  int32_t n_factored;
  int32_t n_supernodes;
  int32_t height;
  int32_t max_front;
  int64_t g_entries;
} cgp_ndchol_info;

/* Factor structure of a context created with CGP_PRECOND_NDCHOL (zeros
 * otherwise). */
int cgp_query_ndchol(const cgp_ctx* ctx, cgp_ndchol_info* out);

/* ---- Lattice mass operator -----------------------------------------------
 * The consistent mass solves (Eqs. 25, 26) run on a lattice layout of the
 * fine nodes: inside a coarse triangle every fine triangle has area
 * |T| / 4^k and edges parallel to T's, so M is applied from the coarse
 * areas and lattice offsets (stored matrix rows only at coarse vertices).
 * Host-only check of that operator on a context: y = M x and diag = M_ii
 * for x (host [N_f], fine numbering), with the rows of the coarse vertices
 * taken from the given CSR matrix (rowptr [N_c + 1] at least, col, mval; fine
 * numbering, columns in range).  Errors: CGP_ERR_INVALID. */
int cgp_lattice_mass_apply_host(const cgp_ctx* ctx, const int32_t* rowptr, const int32_t* col,
                                const double* mval, const double* x, double* y, double* diag);

/* Host-only check of the momentum rows (Eq. 21) that the library assembles
 * on the lattice layout: for host u_prev, u [2][N_f], p [N_f] (may be NULL:
 * no pressure term), u_dir [2][n_dirichlet], f [2][N_f] and t_nat [2][N_f]
 * (may be NULL), fills the rows of the fine nodes other than the coarse
 * vertices: aval [nnz_fine] of A = 3/2 M + dt nu K + dt N(2 U^n - U^{n-1})
 * (identity on Dirichlet rows), rhs [2][N_f], x0 [2][N_f] (the initial guess:
 * W, the boundary values on Dirichlet rows) and r0 [2][N_f] (the initial
 * residual rhs - A x0 that the assembly forms for BiCGSTAB), every other
 * entry NaN; rowptr [N_f + 1] and col [nnz_fine] receive the library's fine
 * CSR structure (diagonal first in each row, then the columns in increasing
 * order).  Errors: CGP_ERR_INVALID (arguments, or a context whose fine rows
 * do not all have the lattice form). */
int cgp_lattice_momentum_host(const cgp_ctx* ctx, const double* u_prev, const double* u,
                              const double* p, const double* u_dir, const double* f,
                              const double* t_nat, int32_t* rowptr, int32_t* col, double* aval,
                              double* rhs, double* x0, double* r0);

/* Host-only check of the right-hand sides of the consistent-mass solves as
 * the library forms them on the lattice layout (fine geometry from the coarse
 * triangles): for host phi_f [N_f] and u_tilde [2][N_f] (fine numbering),
 * rhs [N_f][3] receives -(2/3) dt (G phi_f)_i (0 on velocity-Dirichlet rows)
 * in its first two entries and, for chi = 1, -nu (D U~)_i in the third (0
 * for chi = 0), with G = -D^T and (D U)_i the integral of psi_i div U_h
 * (Eqs. 25-26).  With phi_c [N_c] (not NULL) phi_f is taken to be its
 * prolongation (Eq. 24), the form cgp_project_step uses, and phi_f is not
 * read (may be NULL).  Every index is checked.  Errors: CGP_ERR_INVALID. */
int cgp_lattice_correct_rhs_host(const cgp_ctx* ctx, const double* phi_f, const double* phi_c,
                                 const double* u_tilde, double* rhs);

/* Host-only check of the device mass solves (Eqs. 25-26): a whole solve of
 * `iters` Chebyshev steps from x_0 = 0,
 *   x_{j+1} = x_j + ca_j (x_j - x_{j-1}) + cb_j D^-1 (b - M x_j),
 * (ca_j, cb_j) of the three-term recurrence on [1/2, 2], run launch by launch
 * as the library runs it on lattice size 8: with pairs != 0 the step pairs
 * (a step on the coarse-edge and vertex nodes, the two-step kernel on the
 * interior nodes of the coarse triangles block by block, each phase for
 * every thread before the next, a step on the edge and vertex nodes), with
 * pairs == 0 every step on every node; every index checked.  With
 * mixed != 0 the solve of CGP_MASS_CONSISTENT_MIXED: the sequence above with
 * float-stored iterates on b's float copy (d1), the FP64 residual
 * r = b - M d1 stored as float, the same on r (d2), x = d1 + d2.  Velocity
 * components (0, 1) are 0 at Dirichlet nodes.  b, x: host [N_f][nr], fine
 * numbering, nr 2 or 3; rowptr, col, mval as for
 * cgp_lattice_mass_apply_host.  The iterates start as NaN, so a value read
 * before the sequence wrote it comes back as NaN.  Errors: CGP_ERR_INVALID
 * (arguments, iters outside 1..1000, another lattice size, an index out of
 * range). */
int cgp_lattice_cheb_solve_host(const cgp_ctx* ctx, const int32_t* rowptr, const int32_t* col,
                                const double* mval, int32_t nr, const double* b, int32_t iters,
                                int32_t pairs, int32_t mixed, double* x);

/* Host-only: orders, factors and applies the nested-dissection factor of a
 * symmetric positive definite CSR matrix restricted to the rows/columns with
 * skip[i] == 0: z = K^-1 r there, z = 0 at skipped rows, by the level
 * algorithm of the device solves.  rowptr [n+1], col, val [rowptr[n]]
 * (columns in range, both triangles present), xy [2n] node coordinates
 * (the ordering), skip [n], r and z [n]; all host.  info may be NULL.
 * Errors: CGP_ERR_INVALID (arguments, or a non-positive pivot). */
int cgp_ndchol_solve_host(int32_t n, const int32_t* rowptr, const int32_t* col,
                          const double* val, const double* xy, const uint8_t* skip,
                          const double* r, double* z, cgp_ndchol_info* info);

/* Host-only: the tiling of CGP_PRECOND_JACOBI_S4 for a symmetric CSR graph
 * (rowptr [n+1], col; every row holds its diagonal; xy [2n] node
 * coordinates).  perm [n] receives the internal order (internal index ->
 * node), own_off [n+1] the internal range [own_off[t], own_off[t+1]) of the
 * nodes tile t owns (at most 512), info [4] = (tiles, most nodes a tile owns,
 * largest depth-4 neighbourhood (at most 1024 nodes), ELL width; a tile's
 * rows within distance 3 times the width is at most 7680).  The plan is checked against every
 * invariant the kernels rely on before it is returned.  All host.
 * Errors: CGP_ERR_INVALID (arguments, or a neighbourhood over capacity). */
int cgp_ca_plan_host(int32_t n, const int32_t* rowptr, const int32_t* col, const double* xy,
                     int32_t* perm, int32_t* own_off, int32_t* info);

/* Releases the context's host memory; the workspace and the page-locked
 * host buffer stay the caller's.  Safe on NULL. */
void cgp_destroy(cgp_ctx* ctx);

/* Thread-local description of the last error (never NULL). */
const char* cgp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CGP_H */
