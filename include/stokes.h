/*
 * C ABI of the MI355X matrix-free blended-shell Stokes solver.
 *
 * The operation is the discrete compressible Stokes problem of arXiv
 * 2506.04157, Sec. 5: P2-P1 Taylor-Hood elements on a uniformly refined
 * macro mesh of the unit cube or of the icosahedral hollow sphere, mapped by
 * the radial blending map (Sec. 4.1), with blocks
 *   A_ij = int 2 eta [eps(phi_j):eps(phi_i) - div phi_j div phi_i / 3]
 *   B_ij = - int div phi_j psi_i,   C_ij = - int (grad ln rho . phi_j) psi_i
 * (Sec. 5.1; eta in the divergence term, as the deviatoric stress of Sec. 2
 * implies), solved by FGMRES right-preconditioned with the symmetric Uzawa
 * block preconditioner (eq. SymmetricUzawaStep1), whose A-block inverse is a
 * CG preconditioned by a Chebyshev-smoothed geometric multigrid V-cycle
 * (Sec. 5.2.2) and whose Schur inverse is the V-cycle BFBT approximation
 * (eq. schurV, Sec. 5.2.3).
 *
 * Conventions (all entry points):
 *  - Return 0 on success or a negative STK_E* code; stk_last_error() gives a
 *    thread-local message.  No C++ exception crosses the ABI.
 *  - Vector arguments are caller-owned DEVICE pointers, contiguous, never
 *    freed or kept by the library.  Velocity vectors hold 3*n_p2 values,
 *    component-major [x | y | z], in the library's node order; pressure-type
 *    vectors hold n_p1 values.  "prec" selects the element type of void*
 *    vectors: 64 = double, 32 = float.
 *  - Node order is exposed only through stk_coords; callers match nodes by
 *    coordinates.
 *  - All GPU work is enqueued on the stream given to stk_create; calls that
 *    return host values (sizes, coordinates, reports, scalar outputs)
 *    synchronise that stream.
 *  - Workspaces are allocated by the library at stk_create / stk_set_fields
 *    and freed by stk_destroy.  One context per host thread.
 */
#ifndef STOKES_H
#define STOKES_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STK_OK 0
#define STK_EINVAL (-1)    /* bad argument (null, size, level, eta <= 0 or NaN) */
#define STK_ENOMEM (-2)    /* device allocation failed */
#define STK_EHIP (-3)      /* HIP runtime error */
#define STK_ENOCONV (-4)   /* solver stopped at max iterations; outputs hold the best iterate */
#define STK_ENOTREADY (-5) /* stk_set_fields not called yet */

#define STK_MESH_CUBE 0    /* unit cube split into 6 macro-tets along Kuhn paths */
#define STK_MESH_SHELL 1   /* icosahedral shell: 60 n_tan^2 n_rad macro-tets */

#define STK_BC_DIRICHLET 1 /* prescribed velocity (block row modification, Sec. 5.1) */
#define STK_BC_FREESLIP 2  /* u.n = 0 by projection P_v (Sec. 5.1); shell only */

typedef struct stk_ctx stk_ctx;

typedef struct {
  int kind;            /* STK_MESH_CUBE or STK_MESH_SHELL */
  int n_tan, n_rad;    /* shell: subdivisions of an icosahedron edge, radial layers */
  double r_in, r_out;  /* shell radii (inner, outer) */
  int level;           /* finest refinement level L: 8^L micro-tets per macro-tet */
  int min_level;       /* coarsest multigrid level */
  int bc_inner;        /* BC on r = r_in (cube: on the whole boundary) */
  int bc_outer;        /* BC on r = r_out (shell only) */
} stk_mesh_desc;

/* Solver parameters; stk_default_params fills the values of the paper's
 * Table parametertable plus the readings stated in the comments. */
typedef struct {
  double tol_rel;      /* FGMRES stop: |r| <= tol_rel |b| (Euclidean, projected) */
  double tol_abs;      /* ... or |r| <= tol_abs */
  int restart;         /* FGMRES restart length (not given in the paper) */
  int max_outer;       /* FGMRES iteration cap */
  int precision;       /* 64: all FP64; 32: FP32 preconditioner inside FP64 FGMRES */
  double sigma, omega; /* Uzawa scalings: 1, 0.3 */
  double tol_A;        /* A-block CG relative tolerance: 1e-2 */
  double tol_vbfbt;    /* CG on B Ac^-1 B^T: 1e-1 */
  double tol_invmass;  /* CG on M_{1/eta}: 1e-10 */
  double tol_coarse;   /* coarse-grid CG: 1e-2 */
  int m_A, deg_A;      /* Chebyshev steps / degree in the A-block V-cycle: 3, 2 */
  int m_V, deg_V;      /* ... in the BFBT V-cycle Ac: 1, 1 */
  int max_inner;       /* cap for every inner CG */
  int use_Bbar;        /* 1: B + C in the Uzawa pressure update (eq. SymmetricUzawaStep1 remark) */
  int power_its;       /* power iterations for lambda_max(D^-1 A): 15 */
  double cheb_lo, cheb_hi; /* Chebyshev interval = [cheb_lo, cheb_hi] * lambda_max: 0.12, 1.2 */
  int uzawa;           /* block preconditioner (Sec. 5.2.1): STK_UZAWA_SYMMETRIC (default),
                          STK_UZAWA_INEXACT (eq. InexactUzawaStep1), STK_UZAWA_ADJOINT
                          (eq. AdjointInexactUzawaStep1) */
  int schur;           /* Schur approximation (Sec. 5.2.3): STK_SCHUR_VBFBT (eq. schurV,
                          default), STK_SCHUR_MASS (eq. schurMass, M_{1/eta} CG to
                          tol_invmass), STK_SCHUR_DIAG_BFBT (diag(A)-BFBT: the BFBT form
                          with C = D = diag(A)), STK_SCHUR_WBFBT (the weighted BFBT,
                          eq. schurWBFBT with its Poisson replacements) */
  double a_l, a_r;     /* w-BFBT scalings of eta_l, eta_r near the Dirichlet boundary: 1, 1 */
  double tol_wbfbt;    /* CG on the Poisson operators K_{1/sqrt eta}: 1e-10 (relative or absolute) */
  double tol_vmass;    /* CG on the vector masses M_{sqrt eta}: 1e-4 */
  int initial_guess;   /* 1: stk_solve / stk_solve_adjoint start FGMRES from the values u, p
                          (lu, lp) hold on entry (projected first; in a time loop the previous
                          step's solution, Sec. 6), 0: from zero.  The stop rule is unchanged */
} stk_solver_params;

enum { STK_UZAWA_SYMMETRIC = 0, STK_UZAWA_INEXACT = 1, STK_UZAWA_ADJOINT = 2 };
enum { STK_SCHUR_VBFBT = 0, STK_SCHUR_MASS = 1, STK_SCHUR_DIAG_BFBT = 2, STK_SCHUR_WBFBT = 3 };

typedef struct {
  int iterations;          /* FGMRES iterations */
  double rel_residual;     /* final projected FP64 residual / initial */
  double abs_residual;
  double initial_residual;
  int a_solves, a_cg_its;  /* A-block solves and their total CG iterations */
  int s_solves, s_cg_its;  /* BFBT inner solves and their total CG iterations */
  int vcycles;             /* V-cycles on the finest level */
  int coarse_its;          /* coarse-grid CG iterations (all V-cycles) */
  int mass_its;            /* M_{1/eta} CG iterations (all BFBT solves) */
  double seconds;          /* wall time of the solve (host clock, stream synchronised) */
  int history_len;
  double history[256];     /* relative residual after each FGMRES iteration */
} stk_report;

/* Sec. 4.1 (macro mesh of the hollow icosahedron, structured refinement of
 * every macro-tet into 8^level micro-tets, blending map) and Sec. 5.2.2 (the
 * multigrid hierarchy min_level .. level): build the macro mesh, refine,
 * number the nodes and upload the tables.  The context lives on the HIP
 * device that is current on the calling thread (hipSetDevice before the
 * call; torch.cuda.device(...) in Python); every later call on the context
 * must run with that device current.  `hip_stream` is a hipStream_t of that
 * device (NULL = its default stream).  *out receives a library-owned handle,
 * released by stk_destroy.  STK_EINVAL (before any device call) for a bad
 * descriptor, for a mesh whose P2 or P1 node count reaches 2^31 (the kernels
 * use signed 32-bit node indices), or when the coarsest level has more than
 * 262144 P2 nodes or 596523 micro-tets (its CG keeps the element matrices);
 * STK_ENOMEM when device memory runs out. */
int stk_create(const stk_mesh_desc* desc, void* hip_stream, stk_ctx** out);
/* Frees every device and host resource of the context after synchronising
 * its stream; ctx may be NULL. */
int stk_destroy(stk_ctx* ctx);
/* The paper's solver parameters (App. "Solver Parameters", table
 * parametertable) plus the readings noted in stk_solver_params. */
void stk_default_params(stk_solver_params* p);
/* Message of the last error on the calling thread (valid until the next call). */
const char* stk_last_error(void);

/* Sec. 4.2 (P2 velocity and P1 pressure on the refined mesh; Sec. 7 counts
 * the degrees of freedom with the boundary included): node counts of
 * `level` (min_level..level), N_u = 3 n_p2, N_p = n_p1.  Host outputs,
 * nullable. */
int stk_sizes(const stk_ctx* ctx, int level, int64_t* n_p2, int64_t* n_p1);
/* Sec. 4.1 / 4.2 (the P2 nodes are the vertices and edge midpoints of the
 * unblended micro-tets, mapped by the blending map; the P1 nodes are the
 * vertices): node positions in the library's order.  Host outputs, caller
 * allocated: which = 2 (P2 nodes) or 1 (P1 nodes); xyz: 3*n doubles, node
 * major, physical (blended) coordinates, nullable; flags: n bytes, per node
 * 1 = on r_in / cube boundary, 2 = on r_out, 0 = interior, nullable. */
int stk_coords(const stk_ctx* ctx, int level, int which, double* xyz, uint8_t* flags);

/* Fields on the finest level (device, n_p1 doubles): nodal viscosity eta > 0
 * (P1 interpolant, Sec. 5.2.2) and ln rho (nullable: C = 0).  Injects eta to
 * the coarse levels, computes diag(A) without P_v (Sec. 5.2.2) and the
 * Chebyshev bounds per level (FP64 power iteration). */
int stk_set_fields(stk_ctx* ctx, const double* eta_p1, const double* lnrho_p1, const stk_solver_params* params);
/* Same with eta = exp(m) computed on the device from nodal log-viscosity m. */
int stk_set_log_viscosity(stk_ctx* ctx, const double* m_p1, const double* lnrho_p1, const stk_solver_params* params);
/* The viscosity of the geodynamic model (eq. ViscosityDef) from a P2
 * temperature, with quadrature-point evaluation on the coarse levels
 * (Sec. 5.2.2): eta(x, T) = eta_base(|x|) exp(-E_A T + V_A (r_out - |x|)),
 * eta_base linear between n_base >= 2 samples on a uniform grid of
 * [r_in, r_out] (host array, > 0) and constant outside.  Levels l_eta+1 ..
 * level take the P1 interpolant with vertex values eta(x_V, T(x_V)) (the
 * coarse ones by injection, as in stk_set_fields); levels min_level .. l_eta
 * evaluate eta at the quadrature points from the P2 temperature injected to
 * that level, and apply A with the element-parallel kernel (l_eta <
 * min_level: none).  T_p2: device, n_p2 doubles of the finest level;
 * lnrho_p1 and params as in stk_set_fields.  Errors: STK_EINVAL for a cube
 * mesh, l_eta >= level, a bad eta_base, or non-finite T, E_A, V_A.  A later
 * stk_set_fields / stk_set_log_viscosity returns every level to P1. */
int stk_set_temperature_viscosity(stk_ctx* ctx, const double* T_p2, const double* lnrho_p1, const double* eta_base,
                                  int n_base, double E_A, double V_A, int l_eta, const stk_solver_params* params);

/* Buoyancy right-hand side f_i = int scale T_h r_hat . phi_i (Sec. 5.1,
 * eq. for f with g = -r_hat, unit material factors); T: n_p2 device doubles,
 * f: 3 n_p2 device doubles (overwritten). */
int stk_rhs_buoyancy(stk_ctx* ctx, const double* T_p2, double scale, double* f_u);

/* Operator applies on `level` (Sec. 5.1).  bc bits: 1 = project the input
 * velocity (Dirichlet -> 0, free slip -> tangential), 2 = project the output.
 * Outputs are overwritten. */
int stk_apply_A(stk_ctx* ctx, int level, int prec, const void* x, void* y, int bc);
int stk_apply_B(stk_ctx* ctx, int level, int prec, const void* u, void* q, int with_C, int bc);
int stk_apply_Bt(stk_ctx* ctx, int level, int prec, const void* p, void* y, int with_Ct, int bc);
/* Sec. 5.1 (eq. SaddlePointStructure, the block operator [[A, B^T],
 * [B + C, 0]] FGMRES applies): fused K [u; p] = [A u + B^T p; (B + C) u] on
 * the finest level (transpose=1: [A u + (B + C)^T p; B u]); bc as above for
 * the velocity parts; C needs ln rho.  Outputs overwritten. */
int stk_apply_K(stk_ctx* ctx, int prec, const void* u, const void* p, void* yu, void* yp, int transpose, int bc);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * A-apply of stk_apply_A with the same arguments and result, which allocates
 * nothing.  The sweep's shared-node slots (3 nmacro nsh2 + nmacro nsh1 values
 * of `prec` on `level`, nsh the shared nodes of one macro) live in a fixed
 * device array of STK_NOALLOC_SCRATCH_BYTES that every GPU the library runs
 * on holds until the process ends; a level whose slots need more is refused
 * with STK_EINVAL before any launch.  All calls on one GPU share that array:
 * calls that overlap on one GPU (other streams, threads or contexts) race and
 * give wrong results.  Every call rewrites all the slots it reads, so nothing
 * has to be cleared between calls.  The array's address is looked up once
 * per device by stk_create. */
#define STK_NOALLOC_SCRATCH_BYTES (128u << 20)
int stk_apply_A_noalloc(stk_ctx* ctx, int level, int prec, const void* x, void* y, int bc);
/* P1 mass with weight 1/eta (Sec. 5.2.3, eq. schurMass, M_{1/eta}; the
 * consistent mass with 1/eta_h at the quadrature points): q = M p, p and q
 * n_p1 values of `prec` on `level`; q overwritten. */
int stk_apply_mass(stk_ctx* ctx, int level, int prec, const void* p, void* q);
/* The operators of the weighted BFBT (Sec. 5.2.3, eq. schurWBFBT and the
 * scaled viscosities eta_l, eta_r after it), for parity tests; fields must
 * be set.  a > 0 scales eta by a^2 on the micro-tets that have a vertex on a
 * Dirichlet boundary (the set D_eta).
 * stk_apply_vmass: y = M_{sqrt eta} u on the finest level, the P2 vector mass
 *   with weight sqrt(a^2 eta_h) at the points of a 27-point degree-5 rule;
 *   u, y: 3 n_p2 values of `prec`, y overwritten; bc bits as for A.
 * stk_apply_poisson: q = K_{1/sqrt eta} p on `level`, the P1 Poisson
 *   (Neumann) operator with weight (a^2 eta_h)^{-1/2} (eta injected on the
 *   coarse levels); p, q: n_p1(level) values of `prec`, q overwritten.
 * stk_p1_transfer: the nested P1 prolongation from `level`-1 to `level`
 *   (restrict = 0: in n_p1(level-1) values, out n_p1(level)) or its
 *   transpose (restrict = 1), the transfers of the Poisson multigrid; out
 *   overwritten. */
int stk_apply_vmass(stk_ctx* ctx, int prec, double a, const void* u, void* y, int bc);
int stk_apply_poisson(stk_ctx* ctx, int level, int prec, double a, const void* p, void* q);
int stk_p1_transfer(stk_ctx* ctx, int level, int prec, int restrict_, const void* in, void* out);
/* Sec. 5.2.2 (the Jacobi-Chebyshev smoother uses diag(A)): the diagonal of
 * A on `level` without projections, device output of 3 n_p2 doubles,
 * overwritten. */
int stk_diag_A(stk_ctx* ctx, int level, double* d);
/* Sec. 5.2.2 (Chebyshev smoother of the V-cycle; the paper does not state
 * how its interval is found): the interval [lo, hi] of D^-1 A used on
 * `level`, host outputs.  stk_set_fields computes it as [cheb_lo, cheb_hi]
 * times an FP64 power-iteration estimate of lambda_max(D^-1 A) with the
 * projections applied; stk_set_cheb_bounds overrides it for later fields. */
int stk_cheb_bounds(stk_ctx* ctx, int level, double* lo, double* hi);
int stk_set_cheb_bounds(stk_ctx* ctx, int level, double lo, double hi);
/* `steps` applications of the degree-`degree` Jacobi-Chebyshev polynomial to
 * A x = b on `level` with projections (Sec. 5.2.2); x updated in place.  b
 * and x are expected admissible (projected); x leaves projected. */
int stk_smooth(stk_ctx* ctx, int level, int prec, const void* b, void* x, int degree, int steps);
/* Sec. 5.1 (projections applied in the multigrid prolongation and
 * restriction) and Sec. 5.2.2 (geometric multigrid on the nested levels):
 * the canonical P2 prolongation P from `level`-1 to `level` (the coarse
 * function evaluated at the fine nodes) and its transpose, the restriction,
 * on vectors of `prec`; level > min_level.
 * stk_prolong: ec holds 3 n_p2(level-1) values, ef 3 n_p2(level);
 *   add = 0: ef = P_v P ec (overwritten); add = 1: ef += P_v P ec (the
 *   V-cycle's coarse-grid correction).
 * stk_restrict: rf and tf (nullable) hold 3 n_p2(level) values, rc
 *   3 n_p2(level-1) (overwritten); tf = NULL: rc = P_v P^T rf; otherwise
 *   rc = P_v P^T P_v (rf - tf) (the V-cycle's restriction of the residual
 *   b - A x with t = A x). */
int stk_prolong(stk_ctx* ctx, int level, int prec, const void* ec, void* ef, int add);
int stk_restrict(stk_ctx* ctx, int level, int prec, const void* rf, const void* tf, void* rc);
/* Sec. 5.2.2 (Fig. ASolverStructure: V-cycle with Chebyshev pre- and
 * post-smoothing and a coarse-grid CG) and Sec. 5.2.3 (the cheaper cycle A_C
 * inside the V-cycle BFBT): one V-cycle on the finest level from a zero
 * start, x = V(b); which = 0: A-block cycle (m_A, deg_A), 1: BFBT cycle A_C
 * (m_V, deg_V).  b, x: 3 n_p2 values of `prec`, x overwritten. */
int stk_vcycle(stk_ctx* ctx, const stk_solver_params* params, int prec, const void* b, void* x, int which);

/* One application of the block preconditioner chosen in params (uzawa,
 * schur, precision) to the FP64 residual [ru; rp], started from zero, as
 * FGMRES applies it (Sec. 5.2.4): device doubles ru, zu (3 n_p2), rp, zp
 * (n_p1); outputs overwritten, zu projected, zp of arithmetic mean 0.
 * transpose = 1: the preconditioner of K^T (B and B + C swap roles). */
int stk_precondition(stk_ctx* ctx, const stk_solver_params* params, const double* ru, const double* rp, double* zu,
                     double* zp, int transpose);

/* Stokes solve (Sec. 5.2.4): f_u (3 n_p2), g_p (n_p1, nullable = 0),
 * u_dirichlet (3 n_p2, nullable = 0; read at Dirichlet nodes only); outputs
 * u (3 n_p2, includes the Dirichlet values), p (n_p1, arithmetic mean 0).
 * With free slip on both spheres (bc_inner = bc_outer = STK_BC_FREESLIP)
 * the rigid rotations e_k x X are admissible and strain free (Sec. 2), so
 * the solves remove them as P_p removes the pressure constant: u is
 * Euclidean-orthogonal to the three rotation vectors and the residual is
 * measured with their span projected off (the operator entry points apply
 * P_v only).  rep nullable.  Returns STK_ENOCONV with the best iterate if
 * not converged. */
int stk_solve(stk_ctx* ctx, const stk_solver_params* params, const double* f_u, const double* g_p,
              const double* u_dirichlet, double* u, double* p, stk_report* rep);
/* Adjoint of the Stokes solve (the transpose of the system of eq.
 * SaddlePointStructure, solved by the same FGMRES with the preconditioner of
 * K^T): K^T [lu; lp] = [ju; jp] with homogeneous constraints; ju (3 n_p2),
 * jp (n_p1) device doubles in, lu, lp out (overwritten). */
int stk_solve_adjoint(stk_ctx* ctx, const stk_solver_params* params, const double* ju, const double* jp,
                      double* lu, double* lp, stk_report* rep);
/* Gradient of an objective J(u) through the solve, with A of Sec. 5.1 for
 * the viscosity eta_h = sum_k exp(m_k) psi_k (the P1 interpolant of Sec.
 * 5.2.2) and the buoyancy right-hand side f = scale * buoyancy(T) of Sec.
 * 5.1: given the solution u and the adjoint velocity lu (stk_solve_adjoint
 * with ju = dJ/du), g_m[k] = - lu^T (dA/dm_k) u (n_p1) and g_T[i] = lu^T
 * df/dT_i (n_p2); both device doubles, overwritten. */
int stk_gradient(stk_ctx* ctx, const double* u, const double* lu, double scale, double* g_m, double* g_T);

/* Measurement of the A-apply of Sec. 5.1: times `reps` back-to-back
 * A-applies of `level` (input and output projected) between HIP events on
 * the context stream: *ms_apply = average time of the whole operator
 * (plane-sweep kernel, gather of shared nodes, projection); *ms_kernel
 * (nullable) = average time of the plane-sweep kernel alone, launched `reps`
 * more times.  y is overwritten. */
int stk_time_apply_A(stk_ctx* ctx, int level, int prec, const void* x, void* y, int reps, double* ms_apply,
                     double* ms_kernel);
/* Measurement of the A-apply of Sec. 5.1 inside a caller's own timed loop:
 * enable = 1 clears the timer and from then on brackets every plane-sweep
 * kernel of an A-apply on the finest level (stk_apply_A, any precision) with
 * a pair of HIP events on the context stream; enable = 0 stops, waits for
 * the recorded events and returns the summed kernel time in *ms_total and
 * the number of timed launches in *launches (both host, nullable).  At most
 * 4096 launches are timed per enable (later ones are not recorded).
 * Element-parallel levels (2^level <= 2) have no sweep kernel and are not
 * timed. */
int stk_kernel_timer(stk_ctx* ctx, int enable, double* ms_total, int* launches);

/* ---- temperature step (Sec. 3 splitting, Sec. 6 eq. WeakTemp) ------------------
 * The advection-diffusion step of the energy equation on the P2 space of the
 * finest level, FP64 throughout.  With s^{n+1}, s^n, s^{n-1} the variable-step
 * BDF2 weights of Sec. 3 and tau = tau^{n+1}:
 *   L T = s^{n+1} M T + tau [ adv int (u* . grad T) w + int k/(Pe Cp) grad T . grad(w/rho)
 *                             - int Di alpha/Cp T (u* . g) w ],   g = -x/|x|
 *   b   = int (s^n T^n - s^{n-1} T^{n-1}) w
 *         + tau [ int H/Cp w + int Pe Di/(Ra rho Cp) 2 eta eps_d(u*):eps_d(u*) w ]
 * with eps_d the deviatoric strain rate, rho = exp(ln rho_h), ln rho_h and
 * eta_h P1 interpolants, integrals on the 27-point conical-product rule.
 * `adv` weights the advection term that eq. (WeakTemp) prints beside the
 * traced history values: 0 (default) solves the splitting's advection-free
 * step, 1 the printed equation.  Dirichlet rows: T = T_in on the inner
 * sphere (the whole cube boundary), T_out on the outer sphere.
 * Vectors: device doubles; temperatures n_p2, velocities 3 n_p2
 * (component-major), ln rho and eta n_p1.  ln rho may be NULL (rho = 1). */
typedef struct {
  double tau1, tau0;     /* tau^{n+1}, tau^n (> 0) */
  double k, Pe, Cp, Di, alpha, H, Ra;   /* nondimensional coefficients (Sec. 2) */
  double adv;            /* weight of the advection term in the linear system */
  double T_in, T_out;    /* Dirichlet values */
  double tol_abs;        /* FGMRES stop |b - L T| <= tol_abs on the free rows (tol_T) */
  double tol_cg;         /* relative tolerance of the preconditioner's CG */
  int restart, max_outer, max_cg;
  int stored_S;          /* 1: the CG applies S through element matrices stored for the
                            solve (55 doubles per slot of the finest level's 4^3-cube
                            bricks, about 1.9 slots per micro-tet; used only if that memory
                            is free); 0: matrix-free */
} stk_temp_params;
typedef struct {
  int iterations;           /* FGMRES iterations */
  int cg_its;               /* CG iterations of the preconditioner, summed */
  int converged;
  double initial_residual, abs_residual;
  double ms_mmoc, ms_rhs, ms_solve;   /* host clock, stream synchronised (step only) */
  int stored_S;             /* 1 if the solve used stored element matrices of S */
} stk_temp_report;
/* tau1 = tau0 = 1e-3, k = Pe = Cp = Ra = 1, Di = alpha = H = adv = 0,
 * T_in = 1, T_out = 0, tol_abs = 1e-10 (table parametertable's tol_T),
 * tol_cg = 1e-12 (the paper applies the preconditioner exactly),
 * restart 30, max_outer 300, max_cg 5000, stored_S = 1. */
void stk_temp_default_params(stk_temp_params* p);
#define STK_TEMP_APPLY 0   /* y = L x (no Dirichlet rows) */
#define STK_TEMP_SYM 1     /* y = S x, S = s^{n+1} M + tau k/(Pe Cp) K_{1/rho}: the
                              symmetric mass and diffusion part the preconditioner's CG solves */
#define STK_TEMP_DIAG 2    /* y = diag(S) (x ignored, may be NULL) */
#define STK_TEMP_SYM_STORED 3  /* y = S x through stored element matrices (built by the call) */
/* Operator applies for parity tests: y (n_p2) overwritten, no boundary rows;
 * u_star may be NULL (no velocity). */
int stk_temp_apply(stk_ctx* ctx, const stk_temp_params* p, int mode, const double* u_star, const double* lnrho,
                   const double* x, double* y);
/* b of eq. (WeakTemp) (n_p2, overwritten, no boundary rows) from the traced
 * history values That_n, That_nm1 (n_p2), u_star (3 n_p2, nullable: no
 * heating) and eta (n_p1, the viscosity at the extrapolated temperature;
 * nullable when u_star is NULL). */
int stk_temp_rhs(stk_ctx* ctx, const stk_temp_params* p, const double* u_star, const double* lnrho, const double* eta,
                 const double* That_n, const double* That_nm1, double* b);
/* The modified method of characteristics (Sec. 3): out[i] = F(X_d), X_d the
 * departure point of P2 node i after one step of the classical Runge-Kutta
 * method backwards over tau along u(t - tau + theta tau) = theta u_new +
 * (1 - theta) u_old, the velocity at each stage point and F at X_d
 * evaluated in the micro-tet that contains the point (analytic point
 * location through the blending map).  Points that leave the domain are
 * moved radially onto the shell (clamped onto the cube).  F, out: n_p2
 * (distinct buffers); u_new, u_old: 3 n_p2. */
int stk_mmoc(stk_ctx* ctx, const double* F, const double* u_new, const double* u_old, double tau, double* out);
/* T (n_p2, overwritten): the solution of L T = b with the Dirichlet rows, by
 * FGMRES right-preconditioned with a Jacobi-CG on S (Sec. 6); T_init
 * (nullable) starts the free rows.  STK_ENOCONV if max_outer is reached (T
 * holds the last iterate). */
int stk_temp_solve(stk_ctx* ctx, const stk_temp_params* p, const double* u_star, const double* lnrho,
                   const double* b, const double* T_init, double* T, stk_temp_report* rep);
/* One step of the splitting scheme (Sec. 3): u* = u^n + (u^n - u^{n-1})
 * tau^{n+1}/tau^n (eq. Extrapolation); That^n = MMOC(T^n, u*, u^n, tau^{n+1});
 * That^{n-1} = MMOC(MMOC(T^{n-1}, u^n, u^{n-1}, tau^n), u*, u^n, tau^{n+1})
 * (the characteristic through a node followed back to t^n, then to
 * t^{n-1}); b of eq. (WeakTemp); the Dirichlet solve started from T^n.
 * eta (n_p1) is the viscosity at the extrapolated temperature, supplied by
 * the caller.  T_np1 overwritten; That_n, That_nm1 (nullable) receive the
 * traced values. */
int stk_temperature_step(stk_ctx* ctx, const stk_temp_params* p, const double* T_n, const double* T_nm1,
                         const double* u_n, const double* u_nm1, const double* lnrho, const double* eta,
                         double* T_np1, double* That_n, double* That_nm1, stk_temp_report* rep);

/* One step of the coupled scheme (Sec. 3: the temperature first, then the
 * Stokes problem of eq. StokesSub at the new temperature), on a shell.  With
 * sp->initial_guess = 1 the Stokes solve starts from u_n and p_n (p_n
 * nullable: zero), the previous step's solution, as the paper's time loop
 * does (an absolute tolerance that the updated problem may already meet,
 * Sec. 6).  Steps:
 *  1. T* = T^n + (T^n - T^{n-1}) tau^{n+1}/tau^n (eq. Extrapolation) and the
 *     viscosity eta(x, T*) of the model of eq. ViscosityDef (arguments as in
 *     stk_set_temperature_viscosity), used in the shear heating;
 *  2. T^{n+1} as stk_temperature_step does it (tp);
 *  3. the Stokes fields set to eta(x, T^{n+1}) and ln rho, and u^{n+1},
 *     p^{n+1} from stk_solve (sp) with f = buoyancy_scale * int T^{n+1} r_hat
 *     . phi (stk_rhs_buoyancy), g = 0 and no Dirichlet data.
 * Device vectors: T_n, T_nm1, T_np1 (n_p2), u_n, u_nm1, u_np1 (3 n_p2),
 * p_n, p_np1 and lnrho (n_p1; p_n and lnrho nullable).  The context's fields are left at
 * eta(x, T^{n+1}).  Returns the temperature solve's STK_ENOCONV without
 * solving the Stokes problem, else the Stokes solve's code; trep, srep
 * (nullable) receive both reports. */
int stk_coupled_step(stk_ctx* ctx, const stk_solver_params* sp, const stk_temp_params* tp, const double* eta_base,
                     int n_base, double E_A, double V_A, int l_eta, double buoyancy_scale, const double* lnrho,
                     const double* T_n, const double* T_nm1, const double* u_n, const double* u_nm1,
                     const double* p_n, double* T_np1, double* u_np1, double* p_np1, stk_temp_report* trep,
                     stk_report* srep);

#ifdef __cplusplus
}
#endif
#endif /* STOKES_H */
