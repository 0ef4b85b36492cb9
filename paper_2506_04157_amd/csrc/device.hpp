// Device-side views of one refinement level and kernel launch wrappers.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace stk {

// Brick of TS^3 cubes of the macro's cube lattice per workgroup.
constexpr int TS = 4;
constexpr int B2 = 2 * TS + 1;         // P2 box side
constexpr int B1 = TS + 1;             // P1 box side
constexpr int NB2 = B2 * B2 * B2;
constexpr int NB1 = B1 * B1 * B1;
constexpr int BF = 4 * TS + 1;         // fine P2 box side of a coarse brick (transfers)

// Operator selection for the fused element kernel (F_M: P1 mass with weight 1/eta).
enum { F_A = 1, F_BT = 2, F_B = 4, F_C = 8, F_CT = 16, F_M = 32 };
// Boundary handling: bit 0 project the input velocity, bit 1 the output.
enum { BCM_IN = 1, BCM_OUT = 2 };
// BC action per node class.
enum { ACT_NONE = 0, ACT_DIR = 1, ACT_FS = 2 };

// Plane-sweep tables of a level (see mesh.hpp, Sweep) and gather lists.
struct SweepDev {
  int nstrips, cap2, cap1, nsh2, nsh1;
  const int* strip;    // j0, j1 per strip
  const int2* plist2;  // (packed I | J<<10 | K<<20, slot or -1)
  const int* poff2;    // per strip: m2 + 2 offsets
  const int2* plist1;
  const int* poff1;    // per strip: n + 2 offsets
  const int* elist;    // packed type | px<<3 | py<<13
  const int* eoff;     // per strip: n + 1 offsets
  const int4* etab;    // per element: 2 int4 of LDS ring positions and the type (see mesh.hpp)
  int ne2, ne1;        // plane-list entries per macro (all strips)
  const uint32_t* g2tab;   // [nmacro][ne2] global P2 node of every plane-list entry
  const uint32_t* g1tab;   // [nmacro][ne1] global P1 node of every plane-list entry
};
struct GatherDev {
  int nnodes;
  const uint32_t* node;
  const int* ptr;
  const int* slot;
};

// P1 mass stencil of a level: per-macro rows over the 15 lattice directions
// (the node itself, 7 positive directions and their negatives), assembled
// once per viscosity field; macro-boundary rows are partial and summed by a
// gather.  The per-macro matrix is symmetric, so only the node itself and the
// 7 positive directions are stored: the coefficient of node t in direction
// -d is the one of its neighbour j = t - d in direction d.
constexpr int NDIR1D = 15;
constexpr int NSTORE1 = 8;
struct StencilDev {
  int on;                 // 1: the stencil apply is used for this level
  int nsh;                // slots per macro
  const short* nb;        // [15][nloc1] neighbour local index (nloc1 where absent)
  const int* dst;         // [nloc1] slot of macro-boundary nodes, -1 for macro-interior nodes
  const int* inc_ptr;     // [nloc1 + 1] micro-tets containing each node
  const int2* inc;        // (packed type | px<<3 | py<<13 | pz<<23, vertex | direction codes)
  const double* c64;      // [nmacro][8][nloc1 + 1], last column zero
  const float* c32;
  GatherDev g;
};

// Viscosity model of the geodynamic setup (eq. ViscosityDef):
// eta(x, T) = eta_base(r) exp(-EA T + VA (rout - r)), r = |x|, eta_base linear
// between nbase samples on a uniform grid of [rin, rout], constant outside.
struct ViscDev {
  const double* base;
  int nbase;
  double EA, VA, rin, rout;
};

struct LevelDev {
  int n;                  // P1 lattice side 2^L (P2 side 2n)
  int nloc2, nloc1;       // lattice points per macro
  int nmacro, ntiles;
  int blend;              // 1: radial blending, 0: identity
  long long n2, n1;       // global node counts
  const uint32_t* l2g2;   // nmacro * nloc2
  const uint32_t* l2g1;   // nmacro * nloc1
  const double* geo;      // 16 per macro: v0, E (row-major), g, s0
  const float* geof;
  const double* tinv;     // 60 per macro: per type grad lambda_1..3 rows, |det J_F|
  const float* tinvf;
  const uint8_t* bact;    // 16 per macro: BC action by nonzero-weight mask
  const uint8_t* own;     // 16 per macro: ownership by nonzero-weight mask
  const int* tiles;       // 3 ints per brick origin
  SweepDev sw;
  GatherDev g2, g1;
  int elemwise;           // 1: element-parallel kernel (coarse levels)
  const int* eall;        // all micro-tets of a macro: type | px<<3 | py<<13 | pz<<23
  StencilDev ms;          // P1 mass stencil
  const int4* xtab;       // grid-transfer table with this level as the coarse one (2 int4 per entry)
  const int* xoff;        // per tile: first entry
  int qpv;                // 1: A takes eta at the quadrature points from T2 (element-parallel kernels only)
  const double* T2;       // P2 temperature of this level (qpv)
  const float* T2f;
  ViscDev vm;
};

// Boundary node lists of a level (for vector projections).
struct BcDev {
  int ndir, nfs;
  const uint32_t* dir;    // Dirichlet nodes
  const uint32_t* fs;     // free-slip nodes
  const double* nrm;      // 3 per free-slip node
  const float* nrmf;
};

// ---- launch wrappers (defined in kernels.hip) --------------------------------
// Fused plane-sweep apply; sl2 / sl1 are the slot buffers of the level
// (3 * nmacro * nsh2 and nmacro * nsh1 values).  Outputs are fully written
// (no zero fill needed); bcmode & BCM_OUT projects the velocity output.
// ev0 / ev1 (nullable): events recorded on s right before and after the
// plane-sweep kernel (not around the gather and projection).
template <typename R>
void launch_stokes(int flags, const LevelDev& L, const BcDev& bc, const R* u, const R* p, const R* eta,
                   const R* lnrho, R* yu, R* yp, R* sl2, R* sl1, int bcmode, hipStream_t s,
                   hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// LDS layout of the sweep kernel (byte offsets, 16-byte aligned):
//   sy   [3 cap2][3] double  P2 accumulators             (velocity output)
//   syp  [2 cap1]    double  P1 accumulators             (pressure-type output)
//   s1   [2 cap1][4] R       P1 node: x~ (3), eta
//   sx   [3 cap2][3] R       P2 inputs                   (velocity input)
//   sp, srho [2 cap1] R      P1 inputs p, ln rho
//   sg2  [3 cap2], sg1 [2 cap1] int  global node index, or ~slot for shared nodes
//   sti  [64] R              per-type rows grad lambda_1..3 and |det J_F| of the macro
struct SweepLds {
  unsigned sy, syp, s1, sx, sp, srho, sg2, sg1, sti, total;
};
__host__ __device__ inline unsigned lds_align16(unsigned x) { return (x + 15u) & ~15u; }
__host__ __device__ inline SweepLds sweep_lds(int FL, int cap2, int cap1, int rb) {
  const bool NU = FL & (F_A | F_B | F_C), OU = FL & (F_A | F_BT | F_CT);
  const bool NP = FL & (F_BT | F_CT | F_M), NR = FL & (F_C | F_CT), OP = FL & (F_B | F_C | F_M);
  const unsigned c2 = (unsigned)cap2, c1 = (unsigned)cap1, r = (unsigned)rb;
  SweepLds o;
  unsigned at = 0;
  o.sy = at;
  at = lds_align16(at + (OU ? 9u * c2 * 8u : 0u));
  o.syp = at;
  at = lds_align16(at + (OP ? 2u * c1 * 8u : 0u));
  o.s1 = at;
  at = lds_align16(at + 8u * c1 * r);
  o.sx = at;
  at = lds_align16(at + (NU ? 9u * c2 * r : 0u));
  o.sp = at;
  at = lds_align16(at + (NP ? 2u * c1 * r : 0u));
  o.srho = at;
  at = lds_align16(at + (NR ? 2u * c1 * r : 0u));
  o.sg2 = at;
  at = lds_align16(at + ((NU || OU) ? 3u * c2 * 4u : 0u));
  o.sg1 = at;
  at = lds_align16(at + 2u * c1 * 4u);
  o.sti = at;
  at = lds_align16(at + 64u * r);
  o.total = at;
  return o;
}
// LDS bytes of the sweep kernel for a flag set
size_t sweep_lds_bytes(int flags, int cap2, int cap1, int real_bytes);
template <typename R>
void launch_diag(const LevelDev& L, const R* eta, R* d, hipStream_t s);
template <typename R>
void launch_mass_bricks(const LevelDev& L, const R* eta, const R* p, R* y, hipStream_t s);
void launch_mass_diag(const LevelDev& L, const double* eta, double* y, hipStream_t s);
// assemble the P1 mass stencil coefficients (FP64, and an FP32 copy) from eta
void launch_mass_stencil_build(const LevelDev& L, const double* eta, double* c64, float* c32, hipStream_t s);
// y = M_{1/eta} p with the assembled stencil; slots: nmacro * L.ms.nsh values
template <typename R>
void launch_mass_stencil(const LevelDev& L, const R* p, R* y, R* slots, hipStream_t s);
// y = S p with any stencil of the M_{1/eta} layout (coefficients coef)
template <typename R>
void launch_stencil(const LevelDev& L, const R* coef, const R* p, R* y, R* slots, hipStream_t s);
// LDS bytes of the stencil apply
size_t mass_stencil_lds_bytes(int nloc1, int real_bytes);
// weighted BFBT (eq. schurWBFBT): the P1 Poisson stencil K_{1/sqrt eta} with
// the element factor a2 on the micro-tets touching a Dirichlet boundary
void launch_poisson_stencil_build(const LevelDev& L, const double* eta, double a2, double* c64, float* c32,
                                  hipStream_t s);
// d = diagonal of a P1 stencil (overwritten)
template <typename R>
void launch_stencil_diag(const LevelDev& L, const double* c64, R* d, hipStream_t s);
// nested P1 transfers between levels: ef = P ec, rc = P^T rf (both overwritten)
template <typename R>
void launch_p1_prolong(const LevelDev& Lc, const LevelDev& Lf, const R* ec, R* ef, hipStream_t s);
template <typename R>
void launch_p1_restrict(const LevelDev& Lc, const LevelDev& Lf, const R* rf, R* rc, hipStream_t s);
// 27-point conical-product rule of the vector mass: barycentric points, weights
constexpr int VMASS_NQ = 27;
struct VmassRule {
  double lam[VMASS_NQ][4];
  double w[VMASS_NQ];
};
// y = M_{sqrt eta} u (or its diagonal), y overwritten; bcmode & BCM_IN projects u
template <typename R>
void launch_vmass(const LevelDev& L, const VmassRule& qr, const R* eta, R a2, const R* u, R* y, bool diag, int bcmode,
                  hipStream_t s);
// ---- temperature step (Sec. 3 and Sec. 6, eq. WeakTemp) -----------------------
// Coefficients of the discrete advection-diffusion problem, with tau = tau^{n+1}:
//   L = s1 M + tau (adv Adv(u*) + kap D_rho - cad Adi(u*)),   S = s1 M + tau kap K_{1/rho}
//   b = M (s0 T^n - sm T^{n-1}) + tau (hsrc M 1 + heat W(u*, eta) / rho)
// kap = k/(Pe Cp), cad = Di alpha/Cp, hsrc = H/Cp, heat = Pe Di/(Ra Cp).
struct TempCoef {
  double s1, s0, sm, tau, kap, adv, cad, hsrc, heat;
};
enum { TM_APPLY = 0, TM_SYM = 1, TM_DIAG = 2, TM_RHS = 3 };
// Finest-level element kernel of the temperature problem, 27-point rule:
// TM_APPLY y = L x, TM_SYM y = S x, TM_DIAG y = diag(S), TM_RHS y = b (from
// Tn, Tm, u, eta); no boundary rows (y overwritten).  u (3 n2, component
// major) and lnrho (P1) are nullable (zero velocity, rho = 1).
void launch_temp(const LevelDev& L, const VmassRule& qr, const TempCoef& tc, int mode, const double* x,
                 const double* u, const double* lnrho, const double* eta, const double* Tn, const double* Tm, double* y,
                 hipStream_t s);
// S = s1 M + tk K_{1/rho} as stored element matrices (55 doubles per brick
// slot: nmacro * ntiles * 384 slots of the finest level's bricks, entry-major),
// and y = S x with them (y overwritten).
constexpr int TEMP_SMAT_ENTRIES = 55;
size_t temp_smat_slots(const LevelDev& L);
void launch_temp_smat(const LevelDev& L, const VmassRule& qr, double s1, double tk, const double* lnrho, double* S,
                      hipStream_t s);
void launch_temp_sapply(const LevelDev& L, const double* S, const double* x, double* y, hipStream_t s);
// Point location in the blended mesh.  Shell: the icosahedral face whose cone
// holds the direction (fmat: inverse of the face's vertex matrix), the
// sub-triangle of its n_tan lattice, the radial layer, and among the prism's
// three macro-tets the one containing the inverse-blended point; cube: the
// best of the six macro-tets.  Then the lattice cube and micro-tet type.
struct LocDev {
  int kind;                  // 0 cube, 1 shell
  int n_tan, n_rad;
  double r_in, r_out;
  double fmat[20][9];        // row-major inverse of [v_f0 v_f1 v_f2] (columns)
  double tinv6[6][9];        // row-major inverse of the lattice offsets [o1-o0 o2-o0 o3-o0] of each type
  const int* prism;          // shell: [20][2 n_tan^2][n_rad][3] macro ids
  const double* minv;        // per macro: row-major inverse of E (reference x~ - v0 = E (a, b, c))
};
// out[i] = F(X_d(i)) for every P2 node i of the finest level: X_d the end
// of one classical Runge-Kutta step backwards over tau along the velocity
// linearly interpolated between un (at t) and uo (at t - tau); points that
// leave the domain are moved back onto it (radially on the shell).
void launch_mmoc(const LevelDev& L, const LocDev& loc, const double* F, const double* un, const double* uo, double tau,
                 double* out, hipStream_t s);
// Dirichlet rows of a scalar P2 field on the node list (kind 1 inner / cube, 2 outer):
// set = 0: v = 0 there; set = 1: v = vin / vout there
void launch_scalar_dirichlet(const uint32_t* node, const uint8_t* kind, int nb, double* v, int set, double vin,
                             double vout, hipStream_t s);

// coefficients per level: nmacro * NSTORE1 * (nloc1 + 1)
void launch_rhs(const LevelDev& L, const double* T, double scale, double* f, hipStream_t s);
void launch_gradient(const LevelDev& L, const double* eta, const double* u, const double* lam,
                     double* gm, double* gT, double scale, hipStream_t s);
template <typename R>
void launch_prolong(const LevelDev& Lc, const LevelDev& Lf, const R* ec, R* ef, int bcmode, hipStream_t s);
template <typename R>
void launch_restrict(const LevelDev& Lc, const LevelDev& Lf, const R* rf, R* rc, int bcmode, hipStream_t s);
// ef += P ec (projected as bcmode & BCM_OUT says)
template <typename R>
void launch_prolong_add(const LevelDev& Lc, const LevelDev& Lf, const R* ec, R* ef, int bcmode, hipStream_t s);
// rc = P^T (bf - tf); rc zero-filled by the caller
template <typename R>
void launch_restrict_diff(const LevelDev& Lc, const LevelDev& Lf, const R* bf, const R* tf, R* rc, int bcmode,
                          hipStream_t s);
template <typename R>
void launch_inject(const LevelDev& Lc, const LevelDev& Lf, const R* vf, R* vc, hipStream_t s);
// P2 nodal values of the next coarser level (coarse node = fine node)
template <typename R>
void launch_inject_p2(const LevelDev& Lc, const LevelDev& Lf, const R* vf, R* vc, hipStream_t s);
// P1 viscosity eta(x_V, T(x_V)) at the vertices of level L from its P2 temperature L.T2
void launch_eta_vertices(const LevelDev& L, double* eta1, hipStream_t s);
// diag(A) (no projection) summed from the element matrices' diagonals; d zeroed by the caller
void launch_elem_diag(const LevelDev& L, const double* eta, double* d, hipStream_t s);
template <typename R>
void launch_project(const BcDev& bc, long long n2, R* v, hipStream_t s);

// vector kernels
template <typename R> void vfill(R* x, R a, long long n, hipStream_t s);
template <typename R> void vcopy(const R* x, R* y, long long n, hipStream_t s);
template <typename R> void vaxpy(R a, const R* x, R* y, long long n, hipStream_t s);        // y += a x
template <typename R> void vaxpby(R a, const R* x, R b, R* y, long long n, hipStream_t s);  // y = a x + b y
template <typename R> void vscale(R a, R* x, long long n, hipStream_t s);
template <typename R> void vmul(const R* a, const R* x, R* y, long long n, hipStream_t s);  // y = a .* x
template <typename A, typename B> void vconvert(const A* x, B* y, long long n, hipStream_t s);
template <typename R> void vinvert(const R* d, R* y, long long n, hipStream_t s);          // y = 1/d (0 -> 1)
void vexp(const double* x, double* y, long long n, hipStream_t s);
// Chebyshev smoother updates; xin = false: x enters as zero and is not read.
// r = b - t (t nullable: r = b); d = c1 dinv .* r
template <typename R> void vcheb_start(const R* b, const R* t, const R* dinv, R c1, R* r, R* d, long long n, hipStream_t s);
// one degree-1 step: x += c1 dinv .* (b - t) (t nullable)
template <typename R> void vcheb_one(const R* b, const R* t, const R* dinv, R c1, R* x, bool xin, long long n, hipStream_t s);
// r -= t; x += d; d = c1 dinv .* r + c2 d
template <typename R> void vcheb_step(const R* t, const R* dinv, R c1, R c2, R* r, R* x, R* d, bool xin, long long n, hipStream_t s);
// the last step of a degree: x += d + (c1 dinv .* (r - t) + c2 d)
template <typename R> void vcheb_last(const R* t, const R* dinv, R c1, R c2, const R* r, const R* d, R* x, bool xin, long long n, hipStream_t s);
template <typename R> void vsub(const R* b, const R* t, R* r, long long n, hipStream_t s);   // r = b - t
// Deterministic two-stage dot product accumulated in FP64; result to device *out.
template <typename R> void vdot(const R* x, const R* y, long long n, double* partial, double* out, hipStream_t s);
// x += a p; r += b q; *out = |r|^2 (FP64, deterministic, same partial layout as vdot)
template <typename R>
void vaxpy2_nrm(R a, const R* p, R* x, R b, const R* q, R* r, long long n, double* partial, double* out, hipStream_t s);
void vsum_partials(double* partial, int np, double* out, hipStream_t s);

// Removal of the rigid rotations e_k x X from a finest-level velocity (free
// slip on both spheres): X the node positions (node-major, 3 per P2 node),
// gi the inverse of G = sum_i (|X_i|^2 I - X_i X_i^T) (row-major)
struct RotDev {
  const double* X;
  double gi[9];
};
// v -= mean(v) without a host round trip; partial: DOT_BLOCKS doubles
template <typename R>
void launch_remove_mean(R* v, long long n, double* partial, hipStream_t s);
// v -= (G^-1 m) x X with m = sum_i X_i x v_i; partial: 3 * DOT_BLOCKS doubles
template <typename R>
void launch_rot_remove(const RotDev& rd, long long n2, R* v, double* partial, hipStream_t s);

// Fixed device array (per GPU) holding the shared-node slots of the
// allocation-free A-apply; its size in bytes equals STK_NOALLOC_SCRATCH_BYTES.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)128 << 20;
// Looks up the array's address on `device` (which must be current) once and
// keeps it; call at context creation.
hipError_t noalloc_scratch_init(int device);
// The array's address on `device`, or nullptr before noalloc_scratch_init.
void* noalloc_scratch(int device);
constexpr int DOT_BLOCKS = 1024;
// device-resident Jacobi CG pieces (scalars in sc[], partial sums in part[],
// 5 * DOT_BLOCKS doubles; iteration i uses parity i & 1: see kernels.hip)
enum { CGS_RZ = 0, CGS_RR, CGS_THR, CGS_DONE, CGS_IT, CGS_ALPHA, CGS_BETA, CGS_N };
template <typename R>
void cg_init(const R* r, const R* dinv, R* z, long long n, double tol, double* part, double* sc, hipStream_t s);
template <typename R>
void cg_dot(const R* p, const R* q, long long n, double* part, const double* sc, hipStream_t s);
template <typename R>
void cg_update(const R* p, const R* q, const R* dinv, R* x, R* r, R* z, long long n, double* part, const double* sc,
               int parity, hipStream_t s);
template <typename R>
void cg_pupdate(const R* z, R* p, long long n, double* part, double* sc, int parity, hipStream_t s);

// Coarsest-level operator held as element matrices, and the node-based data of
// its CG (FP64).  Vectors are component-major (3 * nn).
struct CoarseDev {
  int ne;                  // micro-tets of the level
  int nn;                  // P2 nodes
  const uint32_t* enode;   // 10 global P2 nodes per element (local node order of the element kernels)
  const double* emat;      // 900 per element: A_e column-major, local DoF index c * 10 + a
  const float* ematf;      // the same rounded to FP32 (coarse solves of the FP32 preconditioner)
  const int* iptr;         // per node: its incidences (element, local node) are slots iptr[i] .. iptr[i+1]-1
  const int* epos;         // per element and local node (e * 10 + a): its incidence slot
  const uint8_t* act;      // per node: ACT_NONE, ACT_DIR or ACT_FS
  const double* nrm;       // 3 per node: free-slip normal (0 elsewhere)
  const double* dinv;      // inverse diagonal of A, 3 * nn
};
constexpr int CCG_ELEMS = 8;   // elements per workgroup of the element kernel (30 threads each)
// A_e of every micro-tet of level L (eta: P1 nodal, FP64), in FP64 and FP32
void launch_elem_matrix(const LevelDev& L, const double* eta, double* emat, float* ematf, hipStream_t s);
// CG on the coarsest level: x = 0, r = P b, z = P D^-1 r, partials and scalars
void ccg_init(const CoarseDev& cd, const double* b, double* x, double* r, double* z, double tol, double* part,
              double* sc, hipStream_t s);
// iteration `it` (0-based): p = z + beta p (p = z at it 0), q = P A p (as
// P A z + beta q), x += alpha p, r -= alpha q, z = P D^-1 r; Y: 30 doubles per
// element, stored by incidence slot (component c at slot + c * 10 ne); fp32:
// products with the FP32 element matrices (FP64 accumulation)
void ccg_iter(const CoarseDev& cd, bool fp32, double* x, double* r, double* z, double* p, double* q, double* Y,
              double* part, double* sc, int it, hipStream_t s);

}  // namespace stk
