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

// Operator selection for the fused Stokes element kernel.
enum { F_A = 1, F_BT = 2, F_B = 4, F_C = 8, F_CT = 16 };
// Boundary handling: bit 0 project the input velocity, bit 1 the output.
enum { BCM_IN = 1, BCM_OUT = 2 };
// BC action per node class.
enum { ACT_NONE = 0, ACT_DIR = 1, ACT_FS = 2 };

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
template <typename R>
void launch_stokes(int flags, const LevelDev& L, const R* u, const R* p, const R* eta,
                   const R* lnrho, R* yu, R* yp, int bcmode, hipStream_t s);
template <typename R>
void launch_diag(const LevelDev& L, const R* eta, R* d, hipStream_t s);
template <typename R>
void launch_mass(const LevelDev& L, const R* eta, const R* p, R* y, hipStream_t s);
void launch_mass_diag(const LevelDev& L, const double* eta, double* y, hipStream_t s);
void launch_rhs(const LevelDev& L, const double* T, double scale, double* f, hipStream_t s);
void launch_gradient(const LevelDev& L, const double* eta, const double* u, const double* lam,
                     double* gm, double* gT, double scale, hipStream_t s);
template <typename R>
void launch_prolong(const LevelDev& Lc, const LevelDev& Lf, const R* ec, R* ef, int bcmode, hipStream_t s);
template <typename R>
void launch_restrict(const LevelDev& Lc, const LevelDev& Lf, const R* rf, R* rc, int bcmode, hipStream_t s);
template <typename R>
void launch_inject(const LevelDev& Lc, const LevelDev& Lf, const R* vf, R* vc, hipStream_t s);
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
// Chebyshev helpers (see solver): d = c1 * Dinv .* r  + c2 * d
template <typename R> void vcheb_dir(const R* dinv, const R* r, R c1, R c2, R* d, long long n, hipStream_t s);
// Deterministic two-stage dot product accumulated in FP64; result to device *out.
template <typename R> void vdot(const R* x, const R* y, long long n, double* partial, double* out, hipStream_t s);
void vsum_partials(double* partial, int np, double* out, hipStream_t s);
constexpr int DOT_BLOCKS = 1024;

}  // namespace stk
