// HIP kernels for gfx950: matrix-free blended P2-P1 Stokes operators,
// grid transfers, adjoint gradient and vector operations.
//
// Operators (Sec. 5.1 of arXiv 2506.04157, with the divergence term of A
// weighted by eta as the deviatoric stress tau = 2 eta (sym grad u - div u I/3)
// of Sec. 2 implies):
//   A:  y_{a,c} = sum_K sum_q W_q 2 eta_h [eps(u):eps(phi_{a,c}) - div u div phi_{a,c}/3]
//   B:  q_i     = - sum_K sum_q W_q psi_i div u
//   C:  q_i     = - sum_K sum_q W_q psi_i (grad ln rho_h . u)
//   B^T, C^T the transposes.
// Integrals are pulled back through the blending map B(x) = s(x) x/|x|
// (s affine per macro-tet, Sec. 4.1) whose Jacobian is recomputed in closed
// form at every quadrature point:  J_B = d g^T + alpha (I - d d^T) with
// d = x/|x|, alpha = s/|x|, g = grad s;  det J_B = alpha^2 (g.d);
// J_B^{-1} = I/alpha + d h^T with h = (d - g/alpha)/(g.d).
// Quadrature: symmetric 4-point rule of degree 2 (the paper does not state
// its rule; this reading keeps the Taylor-Hood rates and positive weights).
//
// Work decomposition of the operator applies (k_sweep): one workgroup per
// (macro-tet, strip of the macro's lattice rows) sweeps the micro-tet layers
// along the macro's third lattice direction, with a ring of P2 and P1 planes
// staged in LDS; each lane takes one micro-tet of the current layer at a time
// and adds its element result to FP64 LDS accumulators.  Completed planes are
// written out: nodes that only this workgroup touches with plain stores, nodes
// shared with other macros or strips into per-macro slots that k_gather sums
// in a fixed order (no global atomics).  The coarsest levels (2^level <= 2)
// use k_elemwise, one thread per micro-tet with global atomics.  diag(A), the
// M_{1/eta} brick kernel, the right-hand side and the gradient work on bricks
// of 4^3 lattice cubes staged in LDS.
#include <mutex>

#include "device.hpp"

namespace stk {

// ---- constants -------------------------------------------------------------
#define QA 0.58541019662496845446    // (5 + 3 sqrt 5)/20
#define QB 0.13819660112501051518    // (5 - sqrt 5)/20
#define QW (1.0 / 24.0)
#define KAP (4.0 * (QA - QB))          // d/dlambda of the edge/vertex shape functions
#define C1 (4.0 * QB - 1.0)
#define NV_OWN (QA * (2.0 * QA - 1.0))  // vertex function at its own point
#define NV_OTH (QB * (2.0 * QB - 1.0))  // vertex function at another point
#define NE_OWN (4.0 * QA * QB)          // edge function at a point of its vertices
#define NE_OTH (4.0 * QB * QB)

__constant__ int c_toff[6][4][3] = {
    {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}},
    {{0, 1, 0}, {1, 0, 1}, {1, 0, 0}, {1, 1, 0}},
    {{0, 1, 0}, {1, 0, 1}, {1, 1, 0}, {0, 1, 1}},
    {{0, 1, 0}, {1, 0, 1}, {0, 1, 1}, {0, 0, 1}},
    {{0, 1, 0}, {1, 0, 1}, {0, 0, 1}, {1, 0, 0}},
    {{1, 1, 0}, {1, 0, 1}, {0, 1, 1}, {1, 1, 1}},
};

// local edge e = (EV0[e], EV1[e]); node index 4 + e
#define EV0(e) ((e) < 3 ? 0 : ((e) < 5 ? 1 : 2))
#define EV1(e) ((e) == 0 ? 1 : ((e) == 1 ? 2 : ((e) == 2 ? 3 : ((e) == 3 ? 2 : 3))))
__host__ __device__ constexpr int eidx(int i, int j) {
  // node index (4..9) of the edge joining vertices i != j
  return (i < j ? i : j) == 0 ? 3 + (i < j ? j : i) : ((i < j ? i : j) == 1 ? 5 + (i < j ? j : i) : 9);
}
static_assert(eidx(0, 1) == 4 && eidx(2, 0) == 5 && eidx(0, 3) == 6 && eidx(2, 1) == 7 && eidx(1, 3) == 8 &&
                  eidx(3, 2) == 9,
              "edge numbering");

template <typename R> __device__ __forceinline__ const R* geo_of(const LevelDev& L);
template <> __device__ __forceinline__ const double* geo_of<double>(const LevelDev& L) { return L.geo; }
template <> __device__ __forceinline__ const float* geo_of<float>(const LevelDev& L) { return L.geof; }
template <typename R> __device__ __forceinline__ const R* tinv_of(const LevelDev& L);
template <> __device__ __forceinline__ const double* tinv_of<double>(const LevelDev& L) { return L.tinv; }
template <> __device__ __forceinline__ const float* tinv_of<float>(const LevelDev& L) { return L.tinvf; }

// Workgroups are dispatched to the chip's 8 XCDs round-robin by workgroup id,
// and each XCD has its own L2.  Numbering the work items so that XCD x takes a
// contiguous range of them (bijectively, for any grid size) puts neighbouring
// macros, which read the same shared nodes, behind the same L2.
constexpr int NXCD = 8;
__device__ __forceinline__ int xcd_item(int bid, int nwg) {
  const int x = bid % NXCD, loc = bid / NXCD, q = nwg / NXCD, r = nwg % NXCD;
  return x * q + (x < r ? x : r) + loc;
}

// 32-bit lattice arithmetic (side m <= 256: all products fit)
__device__ __forceinline__ int tetc(int s) { return s < 0 ? 0 : (s + 1) * (s + 2) * (s + 3) / 6; }
__device__ __forceinline__ int lloc(int I, int J, int K, int m) {
  const int s = m - K;
  return tetc(m) - tetc(s) + J * (s + 1) - ((J * (J - 1)) >> 1) + I;
}
__device__ __forceinline__ int wmask(int I, int J, int K, int m) {
  return ((m - I - J - K) > 0) | ((I > 0) << 1) | ((J > 0) << 2) | ((K > 0) << 3);
}
// Global index of P2 lattice point (I,J,K) (side m, weight mask `mask`) of
// macro `mac`; l2 is the macro's local-to-global table.  Macro-interior points
// are numbered macro by macro in lattice order, so theirs is closed-form (the
// mesh builder checks this) and needs no table load.
__device__ __forceinline__ size_t p2_gidx(const uint32_t* l2, int mac, int I, int J, int K, int m, int mask) {
  return mask == 15 ? (size_t)mac * (size_t)tetc(m - 4) + (size_t)lloc(I - 1, J - 1, K - 1, m - 4)
                    : (size_t)l2[lloc(I, J, K, m)];
}

// reciprocal and reciprocal square root: hardware approximation refined by
// Newton steps (two in FP64, giving full double accuracy)
__device__ __forceinline__ double rsq(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  y = y * fma(-hx * y, y, 1.5);
  return y;
}
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rcp(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(fma(-x, y, 1.0), y, y);
  y = fma(fma(-x, y, 1.0), y, y);
  return y;
}
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

template <typename R> __device__ __forceinline__ void ldsadd(R* p, R v) { unsafeAtomicAdd(p, v); }
template <typename R> __device__ __forceinline__ void gadd(R* p, R v) { unsafeAtomicAdd(p, v); }

// reference position of P2 lattice point (I,J,K) (side m) of a macro
template <typename R>
__device__ __forceinline__ void lattice_x(const R* G, int I, int J, int K, int m, R x[3]) {
  const R im = R(1) / R(m);
  const R a = R(I) * im, b = R(J) * im, c = R(K) * im;
#pragma unroll
  for (int r = 0; r < 3; ++r) x[r] = G[r] + G[3 + 3 * r] * a + G[4 + 3 * r] * b + G[5 + 3 * r] * c;
}

// project a velocity at a node: Dirichlet -> 0, free slip -> remove normal part
template <typename R>
__device__ __forceinline__ void bc_project(int act, const R* G, int I, int J, int K, int m, R& v0, R& v1, R& v2) {
  if (act == ACT_DIR) {
    v0 = v1 = v2 = R(0);
  } else if (act == ACT_FS) {
    R x[3];
    lattice_x(G, I, J, K, m, x);
    R ri = rsq(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    R n0 = x[0] * ri, n1 = x[1] * ri, n2 = x[2] * ri;
    R dn = v0 * n0 + v1 * n1 + v2 * n2;
    v0 -= dn * n0;
    v1 -= dn * n1;
    v2 -= dn * n2;
  }
}

// Geometry at one quadrature point.
template <typename R, bool BLEND>
struct QGeo {
  R d[3], h[3], ia, W;
  __device__ __forceinline__ void eval(const R* G, const R xq[3], R wdetF) {
    if (BLEND) {
      R r2 = xq[0] * xq[0] + xq[1] * xq[1] + xq[2] * xq[2];
      R ri = rsq(r2);
      d[0] = xq[0] * ri;
      d[1] = xq[1] * ri;
      d[2] = xq[2] * ri;
      R s = G[12] * xq[0] + G[13] * xq[1] + G[14] * xq[2] + G[15];
      R alpha = s * ri;
      ia = rcp(alpha);
      R gd = G[12] * d[0] + G[13] * d[1] + G[14] * d[2];
      R igd = rcp(gd);
#pragma unroll
      for (int k = 0; k < 3; ++k) h[k] = (d[k] - G[12 + k] * ia) * igd;
      W = wdetF * alpha * alpha * gd;
    } else {
      W = wdetF;
    }
  }
  // v^T J_B^{-1}  (row vector times inverse Jacobian) = ia v + (v.d) h
  __device__ __forceinline__ void rowJinv(R v[3]) const {
    if (BLEND) {
      R vd = v[0] * d[0] + v[1] * d[1] + v[2] * d[2];
#pragma unroll
      for (int k = 0; k < 3; ++k) v[k] = ia * v[k] + vd * h[k];
    }
  }
  // J_B^{-1} v = ia v + d (h.v)   (equivalently (J_B^{-T})^T applied on the left)
  __device__ __forceinline__ void Jinv(R v[3]) const {
    if (BLEND) {
      R hv = h[0] * v[0] + h[1] * v[1] + h[2] * v[2];
#pragma unroll
      for (int k = 0; k < 3; ++k) v[k] = ia * v[k] + hv * d[k];
    }
  }
  // J_B^{-T} v = ia v + h (d.v)
  __device__ __forceinline__ void JinvT(R v[3]) const { rowJinv(v); }
};

// ---- viscosity at the quadrature points (Sec. 5.2.2, levels up to l_eta) ----
template <typename R> __device__ __forceinline__ const R* t2_of(const LevelDev& L);
template <> __device__ __forceinline__ const double* t2_of<double>(const LevelDev& L) { return L.T2; }
template <> __device__ __forceinline__ const float* t2_of<float>(const LevelDev& L) { return L.T2f; }

// eq. ViscosityDef at radius r and temperature T
template <typename R>
__device__ __forceinline__ R visc_model(const ViscDev& vm, R r, R T) {
  const int nb = vm.nbase;
  R t = (r - R(vm.rin)) / R(vm.rout - vm.rin) * R(nb - 1);
  t = t < R(0) ? R(0) : (t > R(nb - 1) ? R(nb - 1) : t);
  int i = (int)t;
  if (i > nb - 2) i = nb - 2;
  const R w = t - R(i);
  const R b = (R(1) - w) * R(vm.base[i]) + w * R(vm.base[i + 1]);
  return b * exp(-R(vm.EA) * T + R(vm.VA) * (R(vm.rout) - r));
}

// Viscosity at the element's 4 quadrature points from its 10 P2 temperatures,
// returned as the nodal values whose P1 interpolant takes exactly those values
// at the points (the element kernels evaluate eta only there): with Q_q the
// point values and S their sum, v_q = (Q_q - QB S) / (QA - QB), since the
// interpolant at point q is QB sum(v) + (QA - QB) v_q and QA + 3 QB = 1.
// xv: reference vertex positions; the radius of the blended point is s(x).
template <typename R>
__device__ __forceinline__ void qp_viscosity(const ViscDev& vm, const R* G, const R xv[4][3], const R T10[10],
                                             R et[4]) {
  R xs[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) xs[k] = xv[0][k] + xv[1][k] + xv[2][k] + xv[3][k];
  const R tv = T10[0] + T10[1] + T10[2] + T10[3];
  const R te = T10[4] + T10[5] + T10[6] + T10[7] + T10[8] + T10[9];
  const R tq_e[4] = {T10[4] + T10[5] + T10[6], T10[4] + T10[7] + T10[8], T10[5] + T10[7] + T10[9],
                     T10[6] + T10[8] + T10[9]};
  R eq[4], se = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    R xq[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) xq[k] = R(QB) * xs[k] + R(QA - QB) * xv[q][k];
    const R r = G[12] * xq[0] + G[13] * xq[1] + G[14] * xq[2] + G[15];
    const R Tq = R(NV_OTH) * tv + R(NV_OWN - NV_OTH) * T10[q] + R(NE_OTH) * te + R(NE_OWN - NE_OTH) * tq_e[q];
    eq[q] = visc_model<R>(vm, r, Tq);
    se += eq[q];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) et[q] = (eq[q] - R(QB) * se) * R(1.0 / (QA - QB));
}

// Element context: lattice positions and LDS indices of the 10 P2 / 4 P1 nodes.
struct ElemIdx {
  int n2i[10], n1i[4];
};

__device__ __forceinline__ void elem_indices(int type, int cx, int cy, int cz, ElemIdx& e) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    int a = cx + c_toff[type][v][0], b = cy + c_toff[type][v][1], c = cz + c_toff[type][v][2];
    e.n1i[v] = a + B1 * (b + B1 * c);
    e.n2i[v] = 2 * a + B2 * (2 * b + B2 * 2 * c);
  }
#pragma unroll
  for (int ed = 0; ed < 6; ++ed) {
    const int i = EV0(ed), j = EV1(ed);
    int a = 2 * cx + c_toff[type][i][0] + c_toff[type][j][0];
    int b = 2 * cy + c_toff[type][i][1] + c_toff[type][j][1];
    int c = 2 * cz + c_toff[type][i][2] + c_toff[type][j][2];
    e.n2i[4 + ed] = a + B2 * (b + B2 * c);
  }
}

// reference positions of the element's 4 vertices
template <typename R>
__device__ __forceinline__ void elem_vertices(const R* G, int type, int px, int py, int pz, int n, R xv[4][3]) {
  const R in = R(1) / R(n);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    R a = R(px + c_toff[type][v][0]) * in, b = R(py + c_toff[type][v][1]) * in,
      c = R(pz + c_toff[type][v][2]) * in;
#pragma unroll
    for (int r = 0; r < 3; ++r) xv[v][r] = G[r] + G[3 + 3 * r] * a + G[4 + 3 * r] * b + G[5 + 3 * r] * c;
  }
}

__device__ __forceinline__ int type_limit(int type, int n) {
  return type == 0 ? n - 1 : (type == 5 ? n - 3 : n - 2);
}

// ---- fused Stokes element kernel -------------------------------------------
// Per-element state of the fused kernel.  The quadrature point is a template
// parameter so that every register array is indexed with constants.
template <typename R, bool BLEND, int FL>
struct StokesElem {
  static constexpr bool DA = FL & F_A, DBT = FL & F_BT, DB = FL & F_B, DC = FL & F_C, DCT = FL & F_CT,
                        DM = FL & F_M;
  static constexpr bool NU = DA || DB || DC;
  static constexpr bool NP = DBT || DCT || DM;
  static constexpr bool NE = DA || DM;
  static constexpr bool OU = DA || DBT || DCT;
  static constexpr bool OP = DB || DC || DM;
  static constexpr bool NR = DC || DCT;
  static constexpr bool NEED_G = DA || DB;
  R gl[3][3], wdetF, xv[4][3], xs[3];
  R U[3][10], Ev[3][4], base[3][4];
  R et[4], pp[4], set, spp, grr[3];
  R Sacc[3][4], Dacc[3][4], Eacc[3][6];
  R SV[3], VQ[3][4], SP, DP[4];

  // TI: rows grad lambda_1..3 of the affine micro-tet and |det J_F|;
  // fx(v, k): coordinate k of reference vertex v (used with blending);
  // fu(c, a): velocity component c at local P2 node a;  f1(v, &eta, &p, &rho): P1 values at vertex v
  template <class FX, class FU, class F1>
  __device__ __forceinline__ void load(const R* TI, FX fx, FU fu, F1 f1) {
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int k = 0; k < 3; ++k) gl[r][k] = TI[3 * r + k];
    wdetF = R(QW) * TI[9];
    if (BLEND) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int k = 0; k < 3; ++k) xv[v][k] = fx(v, k);
#pragma unroll
      for (int k = 0; k < 3; ++k) xs[k] = xv[0][k] + xv[1][k] + xv[2][k] + xv[3][k];
    }
    if (NU) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int a = 0; a < 10; ++a) U[c][a] = fu(c, a);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        Ev[c][0] = U[c][4] + U[c][5] + U[c][6];
        Ev[c][1] = U[c][4] + U[c][7] + U[c][8];
        Ev[c][2] = U[c][5] + U[c][7] + U[c][9];
        Ev[c][3] = U[c][6] + U[c][8] + U[c][9];
#pragma unroll
        for (int i = 0; i < 4; ++i) base[c][i] = R(C1) * U[c][i] + R(4.0 * QB) * Ev[c][i];
      }
    }
    set = 0;
    spp = 0;
    R rho[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      R ev = 0, pv = 0, rv = 0;
      f1(v, ev, pv, rv);
      if (NE) { et[v] = ev; set += ev; }
      if (NP) { pp[v] = pv; spp += pv; }
      if (NR) rho[v] = rv;
    }
    if (NR) {
#pragma unroll
      for (int k = 0; k < 3; ++k)
        grr[k] = (rho[1] - rho[0]) * gl[0][k] + (rho[2] - rho[0]) * gl[1][k] + (rho[3] - rho[0]) * gl[2][k];
    }
    if (OU) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int i = 0; i < 4; ++i) Sacc[c][i] = 0;
#pragma unroll
        for (int k = 0; k < 6; ++k) Eacc[c][k] = 0;
        SV[c] = 0;
      }
    }
    SP = 0;
  }

  template <int q>
  __device__ __forceinline__ void qp(const R* G) {
    R xq[3];
    if (BLEND) {
#pragma unroll
      for (int k = 0; k < 3; ++k) xq[k] = R(QB) * xs[k] + R(QA - QB) * xv[q][k];
    }
    QGeo<R, BLEND> geo;
    geo.eval(G, xq, wdetF);
    const R W = geo.W;
    // physical gradients of the barycentric coordinates 1..3: J_B^{-T} grad~ lambda_i
    R Lg[3][3];
    if (NEED_G || DA || DBT) {
#pragma unroll
      for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int k = 0; k < 3; ++k) Lg[i][k] = gl[i][k];
        geo.JinvT(Lg[i]);
      }
    }
    R Gm[3][3];
    if (NEED_G) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        R g4[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) g4[i] = base[c][i] + R(KAP) * (i == q ? U[c][i] : U[c][eidx(i, q)]);
#pragma unroll
        for (int k = 0; k < 3; ++k)
          Gm[c][k] = (g4[1] - g4[0]) * Lg[0][k] + (g4[2] - g4[0]) * Lg[1][k] + (g4[3] - g4[0]) * Lg[2][k];
      }
    }
    R pq = 0;
    if (NP) pq = R(QB) * spp + R(QA - QB) * pp[q];
    if (DA || DBT) {
      R S[3][3];
      if (DA) {
        const R e2 = R(2) * (R(QB) * set + R(QA - QB) * et[q]) * W;
        const R tr3 = (Gm[0][0] + Gm[1][1] + Gm[2][2]) * R(1.0 / 3.0);
        S[0][0] = e2 * (Gm[0][0] - tr3);
        S[1][1] = e2 * (Gm[1][1] - tr3);
        S[2][2] = e2 * (Gm[2][2] - tr3);
        S[0][1] = S[1][0] = R(0.5) * e2 * (Gm[0][1] + Gm[1][0]);
        S[0][2] = S[2][0] = R(0.5) * e2 * (Gm[0][2] + Gm[2][0]);
        S[1][2] = S[2][1] = R(0.5) * e2 * (Gm[1][2] + Gm[2][1]);
      } else {
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int k = 0; k < 3; ++k) S[c][k] = 0;
      }
      if (DBT) {
        const R wp = W * pq;
        S[0][0] -= wp;
        S[1][1] -= wp;
        S[2][2] -= wp;
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const R t1 = S[c][0] * Lg[0][0] + S[c][1] * Lg[0][1] + S[c][2] * Lg[0][2];
        const R t2 = S[c][0] * Lg[1][0] + S[c][1] * Lg[1][1] + S[c][2] * Lg[1][2];
        const R t3 = S[c][0] * Lg[2][0] + S[c][1] * Lg[2][1] + S[c][2] * Lg[2][2];
        const R t[4] = {-(t1 + t2 + t3), t1, t2, t3};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          Sacc[c][i] += t[i];
          if (i == q) Dacc[c][i] = t[i];
          else Eacc[c][eidx(i, q) - 4] += t[i];
        }
      }
    }
    if (NR) {
      R gr[3] = {grr[0], grr[1], grr[2]};
      geo.JinvT(gr);
      if (DC) {
        R val = DB ? (Gm[0][0] + Gm[1][1] + Gm[2][2]) : R(0);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const R sv = U[c][0] + U[c][1] + U[c][2] + U[c][3];
          const R se = U[c][4] + U[c][5] + U[c][6] + U[c][7] + U[c][8] + U[c][9];
          const R uq = R(NV_OTH) * sv + R(NV_OWN - NV_OTH) * U[c][q] + R(NE_OTH) * se + R(NE_OWN - NE_OTH) * Ev[c][q];
          val += gr[c] * uq;
        }
        SP += W * val;
        DP[q] = W * val;
      }
      if (DCT) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const R v = -W * pq * gr[c];
          SV[c] += v;
          VQ[c][q] = v;
        }
      }
    }
    if (DB && !DC) {
      const R val = Gm[0][0] + Gm[1][1] + Gm[2][2];
      SP += W * val;
      DP[q] = W * val;
    }
    if (DM) {
      const R v = W * pq / (R(QB) * set + R(QA - QB) * et[q]);
      SP += v;
      DP[q] = v;
    }
  }

  // fo(c, a, value): add to velocity output; f1o(v, value): add to P1 output
  template <class FO, class F1O>
  __device__ __forceinline__ void store(FO fo, F1O f1o) {
    if (OU) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          R y = (DA || DBT) ? (R(C1) * Sacc[c][i] + R(KAP) * Dacc[c][i]) : R(0);
          if (DCT) y += R(NV_OTH) * SV[c] + R(NV_OWN - NV_OTH) * VQ[c][i];
          fo(c, i, y);
        }
#pragma unroll
        for (int ed = 0; ed < 6; ++ed) {
          const int i = EV0(ed), j = EV1(ed);
          R y = (DA || DBT) ? (R(4.0 * QB) * (Sacc[c][i] + Sacc[c][j]) + R(KAP) * Eacc[c][ed]) : R(0);
          if (DCT) y += R(NE_OTH) * SV[c] + R(NE_OWN - NE_OTH) * (VQ[c][i] + VQ[c][j]);
          fo(c, 4 + ed, y);
        }
      }
    }
    if (OP) {
      const R sg = DM ? R(1) : R(-1);   // B and C carry a minus sign
#pragma unroll
      for (int i = 0; i < 4; ++i) f1o(i, sg * (R(QB) * SP + R(QA - QB) * DP[i]));
    }
  }
};


// ---- plane-sweep apply --------------------------------------------------------
// One workgroup sweeps one (macro, strip) along the lattice direction of the
// fourth macro vertex, layer k = 0 .. of micro-tets at a time.  LDS holds a ring
// of three P2 planes (2k, 2k+1, 2k+2) and two P1 planes (k, k+1) of inputs and
// accumulators; after layer k, P2 planes 2k, 2k+1 and P1 plane k are complete
// and are written out while the next planes are staged into their ring slots.
// Nodes that only this workgroup touches get plain stores; shared nodes
// (macro boundary, strip boundary rows) go to slots summed by k_gather.

template <typename R, bool BLEND, int FL>
__global__ __launch_bounds__(256) void k_sweep(LevelDev L, const R* __restrict__ u, const R* __restrict__ p,
                                               const R* __restrict__ eta, const R* __restrict__ lnrho,
                                               R* __restrict__ yu, R* __restrict__ yp, R* __restrict__ sl2,
                                               R* __restrict__ sl1, int bcmode) {
  using E = StokesElem<R, BLEND, FL>;
  constexpr bool NU = E::NU, NP = E::NP, OU = E::OU, OP = E::OP, NR = E::NR, NE = E::NE;
  constexpr bool P2 = NU || OU;
  // accumulators are FP64 for both precisions: LDS FP64 atomic adds are far
  // faster than FP32 ones on this hardware (and more accurate)
  using Acc = double;
  constexpr int NB2 = 4, NB1 = 2;   // plane entries per thread and batch
  // fetch the first loads of the plane traffic ahead (FP32 A-apply only: it
  // is limited to three workgroups per CU by LDS anyway; the other variants
  // would lose occupancy to the extra registers)
  constexpr bool PF = sizeof(R) == 4 && FL == F_A;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const SweepDev& S = L.sw;
  const int cap2 = S.cap2, cap1 = S.cap1;
  const SweepLds lay = sweep_lds(FL, cap2, cap1, sizeof(R));
  Acc* sy = reinterpret_cast<Acc*>(smem_raw + lay.sy);
  Acc* syp = reinterpret_cast<Acc*>(smem_raw + lay.syp);
  R* s1 = reinterpret_cast<R*>(smem_raw + lay.s1);
  R* sx = reinterpret_cast<R*>(smem_raw + lay.sx);
  R* sp = reinterpret_cast<R*>(smem_raw + lay.sp);
  R* srho = reinterpret_cast<R*>(smem_raw + lay.srho);
  int* sg2 = reinterpret_cast<int*>(smem_raw + lay.sg2);
  int* sg1 = reinterpret_cast<int*>(smem_raw + lay.sg1);
  R* sti = reinterpret_cast<R*>(smem_raw + lay.sti);

  const int wid = xcd_item(blockIdx.x, gridDim.x);
  const int strip = wid % S.nstrips;
  const int mac = wid / S.nstrips;
  const int j0 = S.strip[2 * strip];
  const int n = L.n, m2 = 2 * n;
  const int* poff2 = S.poff2 + strip * (m2 + 2);
  const int* poff1 = S.poff1 + strip * (n + 2);
  const int* eoff = S.eoff + strip * (n + 1);
  const uint32_t* G2t = S.g2tab + (size_t)mac * S.ne2;
  const uint32_t* G1t = S.g1tab + (size_t)mac * S.ne1;
  const R* G = geo_of<R>(L) + (size_t)mac * 16;
  const uint8_t* bact = L.bact + (size_t)mac * 16;
  const size_t N2 = (size_t)L.n2;
  const size_t SS2 = (size_t)L.nmacro * S.nsh2;   // slot component stride
  R* ms2 = sl2 + (size_t)mac * S.nsh2;
  R* ms1 = sl1 + (size_t)mac * S.nsh1;
  const int tid = threadIdx.x, bs = blockDim.x;
  const R in = R(1) / R(n);

  auto cnt2 = [&](int K) { return (K >= 0 && K <= m2) ? poff2[K + 1] - poff2[K] : 0; };
  auto cnt1 = [&](int k) { return (k >= 0 && k <= n) ? poff1[k + 1] - poff1[k] : 0; };

  // Plane traffic of one step: P2 planes Kf0/Kf1 are written out and planes
  // Kl0/Kl1 staged into the same ring slots (Kl = Kf mod 3); P1 plane kf is
  // written out and plane kl staged into its slot.  A thread owns a ring
  // position for both the write-out and the staging.  Entries are handled in
  // batches of NB2 (P2) and NB1 (P1) per thread so that each thread issues
  // all its loads of one kind before it waits for any.  The plane-list entry
  // and its global node index (first loads) of the first batch may have been
  // fetched ahead, during the element loop (Pre).
  struct Pre {
    int2 e2[NB2];
    int g2[NB2];
    int2 e1[NB1];
    int g1[NB1];
  };
  struct Counts {
    int f0, f1, c0, c1, n0, nn1, slot0, slot1, tot2, ff, cl, tot1, slotp;
  };
  auto counts = [&](int Kf0, int Kf1, int Kl0, int Kl1, int kf, int kl) {
    Counts q;
    q.f0 = OU ? cnt2(Kf0) : 0;
    q.f1 = OU ? cnt2(Kf1) : 0;
    q.c0 = P2 ? cnt2(Kl0) : 0;
    q.c1 = P2 ? cnt2(Kl1) : 0;
    q.n0 = q.f0 > q.c0 ? q.f0 : q.c0;
    q.nn1 = q.f1 > q.c1 ? q.f1 : q.c1;
    q.slot0 = ((Kl0 >= 0 ? Kl0 : Kf0) % 3) * cap2;
    q.slot1 = ((Kl1 >= 0 ? Kl1 : Kf1) % 3) * cap2;
    q.tot2 = P2 ? q.n0 + q.nn1 : 0;
    q.ff = OP ? cnt1(kf) : 0;
    q.cl = cnt1(kl);
    q.tot1 = q.ff > q.cl ? q.ff : q.cl;
    q.slotp = ((kl >= 0 ? kl : kf) & 1) * cap1;
    return q;
  };
  // plane-list index of the entry a P2 item stages (-1: none)
  auto item2 = [&](const Counts& q, int t, int Kl0, int Kl1, int& pos, int& K, int& q_, bool& b) {
    b = t >= q.n0;
    q_ = b ? t - q.n0 : t;
    pos = (b ? q.slot1 : q.slot0) + q_;
    K = b ? Kl1 : Kl0;
    return (t < q.tot2 && q_ < (b ? q.c1 : q.c0)) ? poff2[K] + q_ : -1;
  };
  auto fetch = [&](Pre& pf, int Kf0, int Kf1, int Kl0, int Kl1, int kf, int kl) {
    const Counts q = counts(Kf0, Kf1, Kl0, Kl1, kf, kl);
#pragma unroll
    for (int i = 0; i < NB2; ++i) {
      int pos, K, qq;
      bool b;
      const int lt = item2(q, i * bs + tid, Kl0, Kl1, pos, K, qq, b);
      pf.e2[i] = lt >= 0 ? S.plist2[lt] : make_int2(0, -1);
      pf.g2[i] = lt >= 0 ? (int)G2t[lt] : -1;
    }
#pragma unroll
    for (int i = 0; i < NB1; ++i) {
      const int t = i * bs + tid;
      const int lt = (t < q.tot1 && t < q.cl) ? poff1[kl] + t : -1;
      pf.e1[i] = lt >= 0 ? S.plist1[lt] : make_int2(0, -1);
      pf.g1[i] = lt >= 0 ? (int)G1t[lt] : -1;
    }
  };
  auto planes = [&](int Kf0, int Kf1, int Kl0, int Kl1, int kf, int kl, const Pre* pre) {
    const Counts q = counts(Kf0, Kf1, Kl0, Kl1, kf, kl);
    for (int base2 = 0, base1 = 0; base2 < q.tot2 || base1 < q.tot1; base2 += NB2 * bs, base1 += NB1 * bs) {
      const bool usepre = pre != nullptr && base2 == 0;
      int pos2[NB2], lt2[NB2], K2[NB2];
      int pos1[NB1], lt1[NB1];
#pragma unroll
      for (int i = 0; i < NB2; ++i) {
        const int t = base2 + i * bs + tid;
        int qq;
        bool b;
        lt2[i] = item2(q, t, Kl0, Kl1, pos2[i], K2[i], qq, b);
        if (OU && t < q.tot2 && qq < (b ? q.f1 : q.f0)) {   // write out the completed node
          const int pos = pos2[i];
          const int g = sg2[pos];
          if (g >= 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) yu[(size_t)g + c * N2] = R(sy[3 * pos + c]);
          } else {
#pragma unroll
            for (int c = 0; c < 3; ++c) ms2[(size_t)(~g) + c * SS2] = R(sy[3 * pos + c]);
          }
        }
      }
#pragma unroll
      for (int i = 0; i < NB1; ++i) {
        const int t = base1 + i * bs + tid;
        pos1[i] = q.slotp + t;
        lt1[i] = -1;
        if (t < q.tot1) {
          const int pos = pos1[i];
          if (OP && t < q.ff) {
            const int g = sg1[pos];
            if (g >= 0) yp[g] = R(syp[pos]);
            else ms1[~g] = R(syp[pos]);
          }
          if (t < q.cl) lt1[i] = poff1[kl] + t;
        }
      }
      // plane-list entries and global node indices (fetched ahead for the first batch)
      int2 en2[NB2], en1[NB1];
      int g2[NB2], g1[NB1];
      if (usepre) {
#pragma unroll
        for (int i = 0; i < NB2; ++i) {
          en2[i] = pre->e2[i];
          g2[i] = pre->g2[i];
        }
#pragma unroll
        for (int i = 0; i < NB1; ++i) {
          en1[i] = pre->e1[i];
          g1[i] = pre->g1[i];
        }
      } else {
#pragma unroll
        for (int i = 0; i < NB2; ++i) {
          en2[i] = lt2[i] >= 0 ? S.plist2[lt2[i]] : make_int2(0, -1);
          g2[i] = lt2[i] >= 0 ? (int)G2t[lt2[i]] : 0;
        }
#pragma unroll
        for (int i = 0; i < NB1; ++i) {
          en1[i] = lt1[i] >= 0 ? S.plist1[lt1[i]] : make_int2(0, -1);
          g1[i] = lt1[i] >= 0 ? (int)G1t[lt1[i]] : 0;
        }
      }
      // values
      R v2[NB2][3], e1v[NB1], p1v[NB1], r1v[NB1];
#pragma unroll
      for (int i = 0; i < NB2; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) v2[i][c] = (NU && lt2[i] >= 0) ? u[(size_t)g2[i] + c * N2] : R(0);
#pragma unroll
      for (int i = 0; i < NB1; ++i) {
        e1v[i] = (NE && lt1[i] >= 0) ? eta[g1[i]] : R(0);
        p1v[i] = (NP && lt1[i] >= 0) ? p[g1[i]] : R(0);
        r1v[i] = (NR && lt1[i] >= 0) ? lnrho[g1[i]] : R(0);
      }
      // into the ring
#pragma unroll
      for (int i = 0; i < NB2; ++i) {
        if (lt2[i] < 0) continue;
        const int pos = pos2[i];
        if (NU) {
          const int I = en2[i].x & 1023, J = (en2[i].x >> 10) & 1023;
          const int mask = wmask(I, J, K2[i], m2);
          if ((bcmode & BCM_IN) && mask != 15) bc_project<R>(bact[mask], G, I, J, K2[i], m2, v2[i][0], v2[i][1], v2[i][2]);
#pragma unroll
          for (int c = 0; c < 3; ++c) sx[3 * pos + c] = v2[i][c];
        }
        if (OU) {
#pragma unroll
          for (int c = 0; c < 3; ++c) sy[3 * pos + c] = 0;
        }
        sg2[pos] = en2[i].y >= 0 ? ~en2[i].y : g2[i];
      }
#pragma unroll
      for (int i = 0; i < NB1; ++i) {
        if (lt1[i] < 0) continue;
        const int pos = pos1[i];
        const int I = en1[i].x & 1023, J = (en1[i].x >> 10) & 1023;
        const R a = R(I) * in, b = R(J) * in, cc = R(kl) * in;
#pragma unroll
        for (int r = 0; r < 3; ++r) s1[4 * pos + r] = G[r] + G[3 + 3 * r] * a + G[4 + 3 * r] * b + G[5 + 3 * r] * cc;
        s1[4 * pos + 3] = e1v[i];
        if (NP) sp[pos] = p1v[i];
        if (NR) srho[pos] = r1v[i];
        if (OP) syp[pos] = 0;
        sg1[pos] = en1[i].y >= 0 ? ~en1[i].y : g1[i];
      }
    }
  };

  // per-type affine data of this macro, and the first planes
  {
    const R* TIg = tinv_of<R>(L) + (size_t)mac * 60;
    for (int i = tid; i < 60; i += bs) sti[i] = TIg[i];
  }
  planes(-1, -1, 0, 1, -1, 0, nullptr);
  planes(-1, -1, 2, -1, -1, 1, nullptr);
  __syncthreads();
  Pre pf;

  const int kmax = n - 1 - j0;
  for (int k = 0; k <= kmax; ++k) {
    // micro-tets of layer k; the next element's table entry is fetched one
    // iteration ahead
    const int e1 = eoff[k + 1];
    int ei = eoff[k] + tid;
    int4 ta = make_int4(0, 0, 0, 0), tb = ta;
    if (ei < e1) {
      ta = S.etab[2 * ei];
      tb = S.etab[2 * ei + 1];
    }
    // first loads of the next plane traffic, in flight during the element loop
    if (PF) fetch(pf, 2 * k, 2 * k + 1, 2 * k + 3, 2 * k + 4, k, k + 2);
    for (; ei < e1; ei += bs) {
      const int4 ca = ta, cb = tb;
      if (ei + bs < e1) {
        ta = S.etab[2 * (ei + bs)];
        tb = S.etab[2 * (ei + bs) + 1];
      }
      const unsigned w[7] = {(unsigned)ca.x, (unsigned)ca.y, (unsigned)ca.z, (unsigned)ca.w,
                             (unsigned)cb.x, (unsigned)cb.y, (unsigned)cb.z};
      int n2i[10], n1i[4];
#pragma unroll
      for (int a = 0; a < 10; ++a) n2i[a] = (a & 1) ? (int)(w[a >> 1] >> 16) : (int)(w[a >> 1] & 0xffffu);
#pragma unroll
      for (int v = 0; v < 4; ++v) n1i[v] = (v & 1) ? (int)(w[5 + (v >> 1)] >> 16) : (int)(w[5 + (v >> 1)] & 0xffffu);
      const int type = cb.w;
      E el;
      el.load(
          sti + type * 10, [&](int v, int r) { return s1[4 * n1i[v] + r]; },
          [&](int c, int a) { return sx[3 * n2i[a] + c]; },
          [&](int v, R& ev, R& pv, R& rv) {
            if (NE) ev = s1[4 * n1i[v] + 3];
            if (NP) pv = sp[n1i[v]];
            if (NR) rv = srho[n1i[v]];
          });
      el.template qp<0>(G);
      el.template qp<1>(G);
      el.template qp<2>(G);
      el.template qp<3>(G);
      el.store([&](int c, int a, R v) { ldsadd(sy + 3 * n2i[a] + c, Acc(v)); },
               [&](int v, R val) { ldsadd(syp + n1i[v], Acc(val)); });
    }
    __syncthreads();
    // write out the completed planes, stage the next ones into their slots
    planes(2 * k, 2 * k + 1, 2 * k + 3, 2 * k + 4, k, k + 2, PF ? &pf : nullptr);
    __syncthreads();
  }
  // last planes (P2 plane 2 kmax + 2, P1 plane kmax + 1)
  planes(2 * kmax + 2, -1, -1, -1, kmax + 1, -1, nullptr);
}

// Element-parallel variant for coarse levels (few micro-tets per macro): one
// thread per micro-tet of the whole mesh, operands gathered from global memory
// and results added with global atomics into zero-filled outputs.
template <typename R, bool BLEND, int FL>
__device__ __forceinline__ void elemwise_one(const LevelDev& L, long long gid, const R* __restrict__ u,
                                             const R* __restrict__ p, const R* __restrict__ eta,
                                             const R* __restrict__ lnrho, R* __restrict__ yu, R* __restrict__ yp,
                                             int bcmode) {
  using E = StokesElem<R, BLEND, FL>;
  const int n = L.n, m2 = 2 * n;
  const int ne = n * n * n;
  const int mac = (int)(gid / ne);
  const int pk = L.eall[gid - (long long)mac * ne];
  const int type = pk & 7, px = (pk >> 3) & 1023, py = (pk >> 13) & 1023, pz = pk >> 23;
  const uint32_t* l2 = L.l2g2 + (size_t)mac * L.nloc2;
  const uint32_t* l1 = L.l2g1 + (size_t)mac * L.nloc1;
  const R* G = geo_of<R>(L) + (size_t)mac * 16;
  const uint8_t* bact = L.bact + (size_t)mac * 16;
  const size_t N2 = (size_t)L.n2;
  int I2[10], J2[10], K2[10];
  size_t g2[10], g1[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int I = px + c_toff[type][v][0], J = py + c_toff[type][v][1], K = pz + c_toff[type][v][2];
    g1[v] = l1[lloc(I, J, K, n)];
    I2[v] = 2 * I;
    J2[v] = 2 * J;
    K2[v] = 2 * K;
  }
#pragma unroll
  for (int ed = 0; ed < 6; ++ed) {
    const int i = EV0(ed), j = EV1(ed);
    I2[4 + ed] = (I2[i] + I2[j]) >> 1;
    J2[4 + ed] = (J2[i] + J2[j]) >> 1;
    K2[4 + ed] = (K2[i] + K2[j]) >> 1;
  }
#pragma unroll
  for (int a = 0; a < 10; ++a) g2[a] = l2[lloc(I2[a], J2[a], K2[a], m2)];
  R xv[4][3];
  if (BLEND) elem_vertices<R>(G, type, px, py, pz, n, xv);
  // quadrature-point viscosity from the P2 temperature (blended shell only)
  R etq[4] = {0, 0, 0, 0};
  const bool qpv = BLEND && E::NE && L.qpv;
  if (qpv) {
    const R* T2 = t2_of<R>(L);
    R T10[10];
#pragma unroll
    for (int a = 0; a < 10; ++a) T10[a] = T2[g2[a]];
    qp_viscosity<R>(L.vm, G, xv, T10, etq);
  }
  // velocity at the 10 nodes, projected once per node (macro-interior nodes need none)
  R uv[10][3];
  if (E::NU) {
#pragma unroll
    for (int a = 0; a < 10; ++a) {
#pragma unroll
      for (int c = 0; c < 3; ++c) uv[a][c] = u[g2[a] + c * N2];
      const int mask = wmask(I2[a], J2[a], K2[a], m2);
      if ((bcmode & BCM_IN) && mask != 15) bc_project<R>(bact[mask], G, I2[a], J2[a], K2[a], m2, uv[a][0], uv[a][1], uv[a][2]);
    }
  }
  E el;
  el.load(
      tinv_of<R>(L) + ((size_t)mac * 6 + type) * 10, [&](int v, int k) { return xv[v][k]; },
      [&](int c, int a) { return uv[a][c]; },
      [&](int v, R& ev, R& pv, R& rv) {
        if (E::NE) ev = qpv ? etq[v] : eta[g1[v]];
        if (E::NP) pv = p[g1[v]];
        if (E::NR) rv = lnrho[g1[v]];
      });
  el.template qp<0>(G);
  el.template qp<1>(G);
  el.template qp<2>(G);
  el.template qp<3>(G);
  el.store([&](int c, int a, R v) { gadd(yu + g2[a] + c * N2, v); }, [&](int v, R val) { gadd(yp + g1[v], val); });
}

template <typename R, bool BLEND, int FL>
__global__ __launch_bounds__(256) void k_elemwise(LevelDev L, const R* __restrict__ u, const R* __restrict__ p,
                                                  const R* __restrict__ eta, const R* __restrict__ lnrho,
                                                  R* __restrict__ yu, R* __restrict__ yp, int bcmode) {
  const long long gid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (gid >= (long long)L.n * L.n * L.n * L.nmacro) return;
  elemwise_one<R, BLEND, FL>(L, gid, u, p, eta, lnrho, yu, yp, bcmode);
}

// sum the slots of shared nodes: P2 vectors (3 components) or P1 scalars
template <typename R, int NC>
__global__ void k_gather(GatherDev gd, const R* __restrict__ sl, size_t sstride, R* __restrict__ y, size_t ystride) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= gd.nnodes) return;
  const int b = gd.ptr[i], e = gd.ptr[i + 1];
  R v[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) v[c] = 0;
  // batches of GB slots: their indices, then their values, are loaded together;
  // the values are still added in slot order
  constexpr int GB = 4;
  for (int k0 = b; k0 < e; k0 += GB) {
    size_t s[GB];
#pragma unroll
    for (int j = 0; j < GB; ++j) s[j] = k0 + j < e ? (size_t)gd.slot[k0 + j] : 0;
    R w[GB][NC];
#pragma unroll
    for (int j = 0; j < GB; ++j)
#pragma unroll
      for (int c = 0; c < NC; ++c) w[j][c] = k0 + j < e ? sl[s[j] + c * sstride] : R(0);
#pragma unroll
    for (int j = 0; j < GB; ++j)
      if (k0 + j < e) {
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c] += w[j][c];
      }
  }
  const size_t g = gd.node[i];
#pragma unroll
  for (int c = 0; c < NC; ++c) y[g + c * ystride] = v[c];
}

// ---- P1 mass stencil of M_{1/eta} (Sec. 5.2.3) --------------------------------
// Assembly: one thread per (macro, local P1 node) sums, over the micro-tets that
// contain the node in a fixed order, the element entries of its row,
//   M_vw = sum_q W_q psi_v(x_q) psi_w(x_q) / eta_h(x_q),
// into the lattice direction of each vertex w.  FP64, no atomics.
template <bool BLEND>
__global__ __launch_bounds__(256) void k_mass_stencil_build(LevelDev L, const double* __restrict__ eta,
                                                            double* __restrict__ c64, float* __restrict__ c32) {
  const int nloc = L.nloc1, n = L.n;
  const long long gid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (gid >= (long long)nloc * L.nmacro) return;
  const int mac = (int)(gid / nloc), t = (int)(gid - (long long)mac * nloc);
  const uint32_t* l1 = L.l2g1 + (size_t)mac * nloc;
  const double* G = L.geo + (size_t)mac * 16;
  double acc[NDIR1D];
#pragma unroll
  for (int d = 0; d < NDIR1D; ++d) acc[d] = 0.0;
  const int k1 = L.ms.inc_ptr[t + 1];
  for (int k = L.ms.inc_ptr[t]; k < k1; ++k) {
    const int2 e = L.ms.inc[k];
    const unsigned ex = (unsigned)e.x;
    const int type = ex & 7, px = (ex >> 3) & 1023, py = (ex >> 13) & 1023, pz = ex >> 23;
    const int v = e.y & 3;
    double et[4], set = 0.0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      et[w] = eta[l1[lloc(px + c_toff[type][w][0], py + c_toff[type][w][1], pz + c_toff[type][w][2], n)]];
      set += et[w];
    }
    const double* TI = L.tinv + ((size_t)mac * 6 + type) * 10;
    const double wdetF = QW * TI[9];
    double xv[4][3], xs[3] = {0.0, 0.0, 0.0};
    if (BLEND) {
      elem_vertices<double>(G, type, px, py, pz, n, xv);
#pragma unroll
      for (int r = 0; r < 3; ++r) xs[r] = xv[0][r] + xv[1][r] + xv[2][r] + xv[3][r];
    }
    double sq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double xq[3] = {0.0, 0.0, 0.0};
      if (BLEND) {
#pragma unroll
        for (int r = 0; r < 3; ++r) xq[r] = QB * xs[r] + (QA - QB) * xv[q][r];
      }
      QGeo<double, BLEND> geo;
      geo.eval(G, xq, wdetF);
      sq[q] = geo.W / (QB * set + (QA - QB) * et[q]);
    }
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      double m = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) m += sq[q] * (v == q ? QA : QB) * (w == q ? QA : QB);
      const int d = (e.y >> (2 + 4 * w)) & 15;
#pragma unroll
      for (int dd = 0; dd < NDIR1D; ++dd)
        if (dd == d) acc[dd] += m;
    }
  }
  // the node itself and the positive directions; a zero column past the end
  // stands for absent neighbours
  const size_t ld = (size_t)nloc + 1;
#pragma unroll
  for (int d = 0; d < NSTORE1; ++d) {
    const size_t o = ((size_t)mac * NSTORE1 + d) * ld + t;
    c64[o] = acc[d];
    c32[o] = (float)acc[d];
    if (t == 0) {
      c64[o + nloc] = 0.0;
      c32[o + nloc] = 0.0f;
    }
  }
}


// Apply: one workgroup per macro stages p of its P1 lattice in LDS and forms
// each row of the stencil (FP64 sums in a fixed order); macro-interior rows
// are final, macro-boundary rows go to slots summed by k_gather.
template <typename R>
__global__ __launch_bounds__(256) void k_mass_stencil(LevelDev L, const R* __restrict__ coef, const R* __restrict__ p,
                                                      R* __restrict__ y, R* __restrict__ sl) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* sp = reinterpret_cast<R*>(smem_raw);
  const int nloc = L.nloc1, mac = xcd_item(blockIdx.x, gridDim.x);
  const size_t ld = (size_t)nloc + 1;
  const uint32_t* l1 = L.l2g1 + (size_t)mac * nloc;
  for (int t = threadIdx.x; t < nloc; t += blockDim.x) sp[t] = p[l1[t]];
  if (threadIdx.x == 0) sp[nloc] = R(0);
  __syncthreads();
  const R* c = coef + (size_t)mac * NSTORE1 * ld;
  for (int t = threadIdx.x; t < nloc; t += blockDim.x) {
    double acc = (double)c[t] * (double)sp[t];
#pragma unroll
    for (int d = 1; d < NSTORE1; ++d) {
      const int jp = L.ms.nb[d * nloc + t], jm = L.ms.nb[(d + 7) * nloc + t];
      acc += (double)c[d * ld + t] * (double)sp[jp];
      acc += (double)c[d * ld + jm] * (double)sp[jm];
    }
    const int slot = L.ms.dst[t];
    if (slot < 0) y[l1[t]] = R(acc);
    else sl[(size_t)mac * L.ms.nsh + slot] = R(acc);
  }
}

// ---- weighted BFBT operators (eq. schurWBFBT) -----------------------------------
// Element factor s_K of the scaled viscosities eta_l, eta_r: a^2 on the
// micro-tets that have a vertex on a Dirichlet boundary, 1 elsewhere.
__device__ __forceinline__ bool touches_dirichlet(const uint8_t* bact, int type, int px, int py, int pz, int n) {
  bool on = false;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int I = px + c_toff[type][v][0], J = py + c_toff[type][v][1], K = pz + c_toff[type][v][2];
    on = on || bact[wmask(I, J, K, n)] == ACT_DIR;
  }
  return on;
}

// The P1 Poisson stencil K_{1/sqrt eta}: per (macro, local P1 node) the row
// sum_K sum_q W_q (s_K eta_h(x_q))^{-1/2} grad psi_v . grad psi_w over the
// micro-tets that contain the node, in the layout of the M_{1/eta} stencil.
// Gradients are the physical ones of the blended element, J_B^{-T} grad lambda.
template <bool BLEND>
__global__ __launch_bounds__(256) void k_poisson_stencil_build(LevelDev L, const double* __restrict__ eta, double a2,
                                                               double* __restrict__ c64, float* __restrict__ c32) {
  const int nloc = L.nloc1, n = L.n;
  const long long gid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (gid >= (long long)nloc * L.nmacro) return;
  const int mac = (int)(gid / nloc), t = (int)(gid - (long long)mac * nloc);
  const uint32_t* l1 = L.l2g1 + (size_t)mac * nloc;
  const double* G = L.geo + (size_t)mac * 16;
  const uint8_t* bact = L.bact + (size_t)mac * 16;
  double acc[NDIR1D];
#pragma unroll
  for (int d = 0; d < NDIR1D; ++d) acc[d] = 0.0;
  const int k1 = L.ms.inc_ptr[t + 1];
  for (int k = L.ms.inc_ptr[t]; k < k1; ++k) {
    const int2 e = L.ms.inc[k];
    const unsigned ex = (unsigned)e.x;
    const int type = ex & 7, px = (ex >> 3) & 1023, py = (ex >> 13) & 1023, pz = ex >> 23;
    const int v = e.y & 3;
    double et[4], set = 0.0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      et[w] = eta[l1[lloc(px + c_toff[type][w][0], py + c_toff[type][w][1], pz + c_toff[type][w][2], n)]];
      set += et[w];
    }
    const double sK = touches_dirichlet(bact, type, px, py, pz, n) ? a2 : 1.0;
    const double* TI = L.tinv + ((size_t)mac * 6 + type) * 10;
    const double wdetF = QW * TI[9];
    double gl[4][3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      gl[1][r] = TI[r];
      gl[2][r] = TI[3 + r];
      gl[3][r] = TI[6 + r];
      gl[0][r] = -(gl[1][r] + gl[2][r] + gl[3][r]);
    }
    double xv[4][3], xs[3] = {0.0, 0.0, 0.0};
    if (BLEND) {
      elem_vertices<double>(G, type, px, py, pz, n, xv);
#pragma unroll
      for (int r = 0; r < 3; ++r) xs[r] = xv[0][r] + xv[1][r] + xv[2][r] + xv[3][r];
    }
    double kv[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double xq[3] = {0.0, 0.0, 0.0};
      if (BLEND) {
#pragma unroll
        for (int r = 0; r < 3; ++r) xq[r] = QB * xs[r] + (QA - QB) * xv[q][r];
      }
      QGeo<double, BLEND> geo;
      geo.eval(G, xq, wdetF);
      const double wq = geo.W / sqrt(sK * (QB * set + (QA - QB) * et[q]));
      double gv[3] = {gl[v][0], gl[v][1], gl[v][2]};
      geo.JinvT(gv);
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        double gw[3] = {gl[w][0], gl[w][1], gl[w][2]};
        geo.JinvT(gw);
        kv[w] += wq * (gv[0] * gw[0] + gv[1] * gw[1] + gv[2] * gw[2]);
      }
    }
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int d = (e.y >> (2 + 4 * w)) & 15;
#pragma unroll
      for (int dd = 0; dd < NDIR1D; ++dd)
        if (dd == d) acc[dd] += kv[w];
    }
  }
  const size_t ld = (size_t)nloc + 1;
#pragma unroll
  for (int d = 0; d < NSTORE1; ++d) {
    const size_t o = ((size_t)mac * NSTORE1 + d) * ld + t;
    c64[o] = acc[d];
    c32[o] = (float)acc[d];
    if (t == 0) {
      c64[o + nloc] = 0.0;
      c32[o + nloc] = 0.0f;
    }
  }
}

// diagonal of a P1 stencil (coefficient of the node itself), summed over the
// macros that share a node: per (macro, local node) an atomic add into a
// zero-filled vector
template <typename R>
__global__ __launch_bounds__(256) void k_stencil_diag(LevelDev L, const double* __restrict__ c64, R* __restrict__ d) {
  const int nloc = L.nloc1;
  const long long gid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (gid >= (long long)nloc * L.nmacro) return;
  const int mac = (int)(gid / nloc), t = (int)(gid - (long long)mac * nloc);
  const double v = c64[(size_t)mac * NSTORE1 * ((size_t)nloc + 1) + t];
  gadd(d + L.l2g1[(size_t)mac * nloc + t], R(v));
}

// lattice point (I, J, K) of local index t on a lattice of side m (inverse of lloc)
__device__ __forceinline__ void lattice_of(int t, int m, int& I, int& J, int& K) {
  K = 0;
  for (;;) {
    const int s = m - K, cnt = (s + 1) * (s + 2) / 2;
    if (t < cnt) break;
    t -= cnt;
    ++K;
  }
  const int s = m - K;
  J = 0;
  for (;;) {
    const int len = s - J + 1;
    if (t < len) break;
    t -= len;
    ++J;
  }
  I = t;
}

// Nested P1 spaces: a fine lattice point is a coarse vertex (all coordinates
// even) or the midpoint of a coarse micro-tet edge, whose direction follows
// from the pattern of odd coordinates (the seven edge directions of the
// refinement: a, b, c, b - a, c - a, c - b and the octahedron diagonal
// a - b + c).  MODE 0: out = P in (fine = coarse vertex value, or the mean of
// the two edge ends); MODE 1: out += P^T in (out zero-filled by the caller).
// One thread per (macro, fine lattice point); each fine node is handled by
// the macro that owns it.
template <typename R, int MODE>
__global__ __launch_bounds__(256) void k_p1_transfer(LevelDev Lc, LevelDev Lf, const R* __restrict__ in,
                                                     R* __restrict__ out) {
  const int nlf = Lf.nloc1, nf = Lf.n, nc = Lc.n;
  const long long gid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (gid >= (long long)nlf * Lf.nmacro) return;
  const int mac = (int)(gid / nlf), t = (int)(gid - (long long)mac * nlf);
  int I, J, K;
  lattice_of(t, nf, I, J, K);
  const int mask = wmask(I, J, K, nf);
  if (Lf.own[(size_t)mac * 16 + mask] == 0) return;
  const size_t gf = Lf.l2g1[(size_t)mac * nlf + t];
  const uint32_t* l2c = Lc.l2g1 + (size_t)mac * Lc.nloc1;
  const int ox = I & 1, oy = J & 1, oz = K & 1;
  if (!(ox | oy | oz)) {
    const size_t gc = l2c[lloc(I >> 1, J >> 1, K >> 1, nc)];
    if (MODE == 0) out[gf] = in[gc];
    else gadd(out + gc, in[gf]);
    return;
  }
  // edge direction by the pattern of odd coordinates: x (1,0,0), y (0,1,0),
  // z (0,0,1), x+y (-1,1,0), x+z (-1,0,1), y+z (0,-1,1), x+y+z (1,-1,1)
  const int dx = ox ? ((oy != oz) ? -1 : 1) : 0;
  const int dy = oy ? (oz ? -1 : 1) : 0;
  const int dz = oz;
  const size_t g0 = l2c[lloc((I - dx) >> 1, (J - dy) >> 1, (K - dz) >> 1, nc)];
  const size_t g1 = l2c[lloc((I + dx) >> 1, (J + dy) >> 1, (K + dz) >> 1, nc)];
  if (MODE == 0) {
    out[gf] = R(0.5) * (in[g0] + in[g1]);
  } else {
    const R h = R(0.5) * in[gf];
    gadd(out + g0, h);
    gadd(out + g1, h);
  }
}

// The P2 vector mass M_{sqrt eta} with weight sqrt(s_K eta_h(x_q)) on the
// 27-point conical-product rule (degree 5; the 4-point rule of the Stokes
// blocks leaves a P2 mass singular).  One thread per micro-tet of the finest
// level; DIAG: the diagonal (same in the three components), else y += M u
// with the input projected (bcmode & BCM_IN) and global atomics into a
// zero-filled y.
template <typename R, bool BLEND, bool DIAG>
__global__ __launch_bounds__(256) void k_vmass(LevelDev L, VmassRule qr, const R* __restrict__ eta, R a2,
                                               const R* __restrict__ u, R* __restrict__ y, int bcmode) {
  const long long gid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int n = L.n, m2 = 2 * n;
  const int ne = n * n * n;
  if (gid >= (long long)ne * L.nmacro) return;
  const int mac = (int)(gid / ne);
  const int pk = L.eall[gid - (long long)mac * ne];
  const int type = pk & 7, px = (pk >> 3) & 1023, py = (pk >> 13) & 1023, pz = pk >> 23;
  const uint32_t* l2 = L.l2g2 + (size_t)mac * L.nloc2;
  const uint32_t* l1 = L.l2g1 + (size_t)mac * L.nloc1;
  const R* G = geo_of<R>(L) + (size_t)mac * 16;
  const uint8_t* bact = L.bact + (size_t)mac * 16;
  const size_t N2 = (size_t)L.n2;
  int I2[10], J2[10], K2[10];
  size_t g2[10];
  R et[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int I = px + c_toff[type][v][0], J = py + c_toff[type][v][1], K = pz + c_toff[type][v][2];
    et[v] = eta[l1[lloc(I, J, K, n)]];
    I2[v] = 2 * I;
    J2[v] = 2 * J;
    K2[v] = 2 * K;
  }
#pragma unroll
  for (int ed = 0; ed < 6; ++ed) {
    const int i = EV0(ed), j = EV1(ed);
    I2[4 + ed] = (I2[i] + I2[j]) >> 1;
    J2[4 + ed] = (J2[i] + J2[j]) >> 1;
    K2[4 + ed] = (K2[i] + K2[j]) >> 1;
  }
#pragma unroll
  for (int a = 0; a < 10; ++a) g2[a] = l2[lloc(I2[a], J2[a], K2[a], m2)];
  const R sK = touches_dirichlet(bact, type, px, py, pz, n) ? a2 : R(1);
  R xv[4][3];
  if (BLEND) elem_vertices<R>(G, type, px, py, pz, n, xv);
  const R* TI = tinv_of<R>(L) + ((size_t)mac * 6 + type) * 10;
  const R detF = TI[9];
  R uv[3][10];
  if (!DIAG) {
#pragma unroll
    for (int a = 0; a < 10; ++a) {
      R v0 = u[g2[a]], v1 = u[g2[a] + N2], v2 = u[g2[a] + 2 * N2];
      const int mask = wmask(I2[a], J2[a], K2[a], m2);
      if ((bcmode & BCM_IN) && mask != 15) bc_project<R>(bact[mask], G, I2[a], J2[a], K2[a], m2, v0, v1, v2);
      uv[0][a] = v0;
      uv[1][a] = v1;
      uv[2][a] = v2;
    }
  }
  R acc[3][10];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int a = 0; a < 10; ++a) acc[c][a] = 0;
  for (int q = 0; q < VMASS_NQ; ++q) {
    const R l0 = R(qr.lam[q][0]), l1 = R(qr.lam[q][1]), l2v = R(qr.lam[q][2]), l3 = R(qr.lam[q][3]);
    const R lam[4] = {l0, l1, l2v, l3};
    R xq[3] = {0, 0, 0};
    if (BLEND) {
#pragma unroll
      for (int r = 0; r < 3; ++r) xq[r] = l0 * xv[0][r] + l1 * xv[1][r] + l2v * xv[2][r] + l3 * xv[3][r];
    }
    QGeo<R, BLEND> geo;
    geo.eval(G, xq, R(qr.w[q]) * detF);
    const R cq = geo.W * sqrt(sK * (l0 * et[0] + l1 * et[1] + l2v * et[2] + l3 * et[3]));
    R N[10];
#pragma unroll
    for (int v = 0; v < 4; ++v) N[v] = lam[v] * (R(2) * lam[v] - R(1));
#pragma unroll
    for (int ed = 0; ed < 6; ++ed) N[4 + ed] = R(4) * lam[EV0(ed)] * lam[EV1(ed)];
    if (DIAG) {
#pragma unroll
      for (int a = 0; a < 10; ++a) acc[0][a] += cq * N[a] * N[a];
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        R uq = 0;
#pragma unroll
        for (int a = 0; a < 10; ++a) uq += N[a] * uv[c][a];
        uq *= cq;
#pragma unroll
        for (int a = 0; a < 10; ++a) acc[c][a] += uq * N[a];
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 10; ++a) {
    if (DIAG) {
      gadd(y + g2[a], acc[0][a]);
      gadd(y + g2[a] + N2, acc[0][a]);
      gadd(y + g2[a] + 2 * N2, acc[0][a]);
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) gadd(y + g2[a] + c * N2, acc[c][a]);
    }
  }
}

// ---- temperature step (Sec. 3 and Sec. 6, eq. WeakTemp) -------------------------
// P2 basis at one point of a micro-tet: the reference point xq, the weight W
// (rule weight times |det J_F| |det J_B|), the physical gradients gL of the
// barycentric coordinates (J_B^{-T} applied to the affine ones), the values N
// and the physical gradients dN of the ten basis functions.
template <bool BLEND>
__device__ __forceinline__ void temp_point(const double* G, const double xv[4][3], const double gl[3][3],
                                           const double lam[4], double wdet, double xq[3], double& W,
                                           double gL[4][3], double N[10], double dN[10][3]) {
#pragma unroll
  for (int r = 0; r < 3; ++r) xq[r] = lam[0] * xv[0][r] + lam[1] * xv[1][r] + lam[2] * xv[2][r] + lam[3] * xv[3][r];
  QGeo<double, BLEND> geo;
  geo.eval(G, xq, wdet);
  W = geo.W;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int k = 0; k < 3; ++k) gL[i + 1][k] = gl[i][k];
    geo.JinvT(gL[i + 1]);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) gL[0][k] = -(gL[1][k] + gL[2][k] + gL[3][k]);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    N[v] = lam[v] * (2.0 * lam[v] - 1.0);
#pragma unroll
    for (int k = 0; k < 3; ++k) dN[v][k] = (4.0 * lam[v] - 1.0) * gL[v][k];
  }
#pragma unroll
  for (int ed = 0; ed < 6; ++ed) {
    const int i = EV0(ed), j = EV1(ed);
    N[4 + ed] = 4.0 * lam[i] * lam[j];
#pragma unroll
    for (int k = 0; k < 3; ++k) dN[4 + ed][k] = 4.0 * (lam[i] * gL[j][k] + lam[j] * gL[i][k]);
  }
}

// Element data of the temperature kernels: the ten global P2 nodes, the four
// P1 nodes' ln rho (0 without), the reference vertices and the affine
// gradients of the barycentric coordinates 1..3 with |det J_F|.
struct TempElem {
  size_t g2[10];
  uint32_t g1[4];
  double xv[4][3], gl[3][3], detF;
  const double* G;
};
__device__ __forceinline__ void temp_elem(const LevelDev& L, int mac, int pk, TempElem& e) {
  const int type = pk & 7, px = (pk >> 3) & 1023, py = (pk >> 13) & 1023, pz = pk >> 23;
  const int n = L.n, m2 = 2 * n;
  const uint32_t* l2 = L.l2g2 + (size_t)mac * L.nloc2;
  const uint32_t* l1 = L.l2g1 + (size_t)mac * L.nloc1;
  e.G = L.geo + (size_t)mac * 16;
  int I2[10], J2[10], K2[10];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int I = px + c_toff[type][v][0], J = py + c_toff[type][v][1], K = pz + c_toff[type][v][2];
    e.g1[v] = l1[lloc(I, J, K, n)];
    I2[v] = 2 * I;
    J2[v] = 2 * J;
    K2[v] = 2 * K;
  }
#pragma unroll
  for (int ed = 0; ed < 6; ++ed) {
    const int i = EV0(ed), j = EV1(ed);
    I2[4 + ed] = (I2[i] + I2[j]) >> 1;
    J2[4 + ed] = (J2[i] + J2[j]) >> 1;
    K2[4 + ed] = (K2[i] + K2[j]) >> 1;
  }
#pragma unroll
  for (int a = 0; a < 10; ++a) e.g2[a] = l2[lloc(I2[a], J2[a], K2[a], m2)];
  elem_vertices<double>(e.G, type, px, py, pz, n, e.xv);
  const double* TI = L.tinv + ((size_t)mac * 6 + type) * 10;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) e.gl[r][k] = TI[3 * r + k];
  e.detF = TI[9];
}

// One thread per micro-tet of the finest level, global atomics, the 27-point
// conical-product rule of the vector mass: the P2 mass integrand has degree
// 4, which the 4-point rule of the Stokes blocks would make singular.  Per
// point: the barycentric coordinates, the P2 values N and physical gradients
// dN (J_B^{-T} applied to the affine gradients), and 1/rho = exp(-ln rho_h).
//   APPLY: y_i += W [N_i (s1 T + tau (adv u.grad T - kap/rho grad ln rho . grad T
//                  - cad (u.g) T)) + tau kap/rho grad T . grad N_i],  g = -X/|X|
//   SYM:   the s1 T N_i and tau kap/rho grad T . grad N_i parts
//   DIAG:  W (s1 N_i^2 + tau kap/rho |grad N_i|^2)
//   RHS:   W N_i (s0 T^n - sm T^{n-1} + tau (hsrc + heat/rho 2 eta eps_d:eps_d))
template <int MODE, bool BLEND>
__global__ __launch_bounds__(256) void k_temp(LevelDev L, VmassRule qr, TempCoef tc, const double* __restrict__ x,
                                              const double* __restrict__ u, const double* __restrict__ lnrho,
                                              const double* __restrict__ eta, const double* __restrict__ Tn,
                                              const double* __restrict__ Tm, double* __restrict__ y) {
  const long long gid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int n = L.n, m2 = 2 * n;
  const int ne = n * n * n;
  if (gid >= (long long)ne * L.nmacro) return;
  const int mac = (int)(gid / ne);
  const int pk = L.eall[gid - (long long)mac * ne];
  const int type = pk & 7, px = (pk >> 3) & 1023, py = (pk >> 13) & 1023, pz = pk >> 23;
  const uint32_t* l2 = L.l2g2 + (size_t)mac * L.nloc2;
  const uint32_t* l1 = L.l2g1 + (size_t)mac * L.nloc1;
  const double* G = L.geo + (size_t)mac * 16;
  const size_t N2 = (size_t)L.n2;
  const bool hasU = u != nullptr && (MODE == TM_APPLY || MODE == TM_RHS);
  int I2[10], J2[10], K2[10];
  size_t g2[10];
  double lr[4], et[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int I = px + c_toff[type][v][0], J = py + c_toff[type][v][1], K = pz + c_toff[type][v][2];
    const uint32_t g1 = l1[lloc(I, J, K, n)];
    lr[v] = lnrho ? lnrho[g1] : 0.0;
    et[v] = (MODE == TM_RHS && eta) ? eta[g1] : 0.0;
    I2[v] = 2 * I;
    J2[v] = 2 * J;
    K2[v] = 2 * K;
  }
#pragma unroll
  for (int ed = 0; ed < 6; ++ed) {
    const int i = EV0(ed), j = EV1(ed);
    I2[4 + ed] = (I2[i] + I2[j]) >> 1;
    J2[4 + ed] = (J2[i] + J2[j]) >> 1;
    K2[4 + ed] = (K2[i] + K2[j]) >> 1;
  }
#pragma unroll
  for (int a = 0; a < 10; ++a) g2[a] = l2[lloc(I2[a], J2[a], K2[a], m2)];
  double xv[4][3];
  elem_vertices<double>(G, type, px, py, pz, n, xv);
  const double* TI = L.tinv + ((size_t)mac * 6 + type) * 10;
  double gl[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) gl[r][k] = TI[3 * r + k];
  const double detF = TI[9];
  double xs[10];
#pragma unroll
  for (int a = 0; a < 10; ++a) {
    if (MODE == TM_APPLY || MODE == TM_SYM) xs[a] = x[g2[a]];
    else if (MODE == TM_RHS) xs[a] = tc.s0 * Tn[g2[a]] - tc.sm * Tm[g2[a]];
    else xs[a] = 0.0;
  }
  double U[3][10];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int a = 0; a < 10; ++a) U[c][a] = hasU ? u[g2[a] + c * N2] : 0.0;
  double acc[10];
#pragma unroll
  for (int a = 0; a < 10; ++a) acc[a] = 0.0;
  for (int q = 0; q < VMASS_NQ; ++q) {
    const double lam[4] = {qr.lam[q][0], qr.lam[q][1], qr.lam[q][2], qr.lam[q][3]};
    double xq[3], W, gL[4][3], N[10], dN[10][3];
    temp_point<BLEND>(G, xv, gl, lam, qr.w[q] * detF, xq, W, gL, N, dN);
    const double irho = exp(-(lam[0] * lr[0] + lam[1] * lr[1] + lam[2] * lr[2] + lam[3] * lr[3]));
    const double tk = tc.tau * tc.kap * irho;
    if (MODE == TM_DIAG) {
#pragma unroll
      for (int a = 0; a < 10; ++a)
        acc[a] += W * (tc.s1 * N[a] * N[a] + tk * (dN[a][0] * dN[a][0] + dN[a][1] * dN[a][1] + dN[a][2] * dN[a][2]));
      continue;
    }
    if (MODE == TM_RHS) {
      double src = tc.tau * tc.hsrc;
#pragma unroll
      for (int a = 0; a < 10; ++a) src += N[a] * xs[a];
      if (hasU) {
        double Gm[3][3];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            double s = 0.0;
#pragma unroll
            for (int a = 0; a < 10; ++a) s += U[c][a] * dN[a][k];
            Gm[c][k] = s;
          }
        const double dv = Gm[0][0] + Gm[1][1] + Gm[2][2];
        double ee = Gm[0][0] * Gm[0][0] + Gm[1][1] * Gm[1][1] + Gm[2][2] * Gm[2][2];
        const double e01 = 0.5 * (Gm[0][1] + Gm[1][0]), e02 = 0.5 * (Gm[0][2] + Gm[2][0]),
                     e12 = 0.5 * (Gm[1][2] + Gm[2][1]);
        ee += 2.0 * (e01 * e01 + e02 * e02 + e12 * e12);
        const double etq = lam[0] * et[0] + lam[1] * et[1] + lam[2] * et[2] + lam[3] * et[3];
        src += tc.tau * tc.heat * irho * 2.0 * etq * (ee - dv * dv * (1.0 / 3.0));
      }
#pragma unroll
      for (int a = 0; a < 10; ++a) acc[a] += W * src * N[a];
      continue;
    }
    double Tq = 0.0, gT[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < 10; ++a) {
      Tq += N[a] * xs[a];
#pragma unroll
      for (int k = 0; k < 3; ++k) gT[k] += dN[a][k] * xs[a];
    }
    double sa = tc.s1 * Tq;
    if (MODE == TM_APPLY) {
      double glr[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) glr[k] = lr[0] * gL[0][k] + lr[1] * gL[1][k] + lr[2] * gL[2][k] + lr[3] * gL[3][k];
      sa -= tk * (glr[0] * gT[0] + glr[1] * gT[1] + glr[2] * gT[2]);
      if (hasU) {
        double uq[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          double s = 0.0;
#pragma unroll
          for (int a = 0; a < 10; ++a) s += N[a] * U[c][a];
          uq[c] = s;
        }
        // the physical point B(x~) lies on the ray of x~: g = -x~/|x~|
        const double ri = rsq(xq[0] * xq[0] + xq[1] * xq[1] + xq[2] * xq[2]);
        const double ug = -(uq[0] * xq[0] + uq[1] * xq[1] + uq[2] * xq[2]) * ri;
        sa += tc.tau * (tc.adv * (uq[0] * gT[0] + uq[1] * gT[1] + uq[2] * gT[2]) - tc.cad * ug * Tq);
      }
    }
    const double b0 = tk * gT[0], b1 = tk * gT[1], b2 = tk * gT[2];
#pragma unroll
    for (int a = 0; a < 10; ++a) acc[a] += W * (sa * N[a] + b0 * dN[a][0] + b1 * dN[a][1] + b2 * dN[a][2]);
  }
#pragma unroll
  for (int a = 0; a < 10; ++a) gadd(y + g2[a], acc[a]);
}

// Stored element matrices of S = s1 M + tau kap K_{1/rho} (the preconditioner's
// operator), built once per solve: the 55 entries i <= j of each micro-tet's
// symmetric 10 x 10 matrix.  Both kernels work on bricks of 4^3 lattice cubes
// (one workgroup per (macro, brick), one wave per micro-tet type, one lane per
// cube), so a micro-tet's slot is ((mac * ntiles + tile) * 6 + type) * 64 + lane
// and the matrices are stored entry-major over these slots (entry e of slot s
// at e * nslots + s): a wave reads each entry coalesced.  Slots of cubes
// outside the macro are left unused.
template <bool BLEND>
__global__ __launch_bounds__(384) void k_temp_smat(LevelDev L, VmassRule qr, double s1, double tk,
                                                   const double* __restrict__ lnrho, double* __restrict__ S) {
  const int wid = xcd_item(blockIdx.x, gridDim.x);
  const int tile = wid % L.ntiles;
  const int mac = wid / L.ntiles;
  const int type = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int px = L.tiles[3 * tile] + (lane & 3), py = L.tiles[3 * tile + 1] + ((lane >> 2) & 3),
            pz = L.tiles[3 * tile + 2] + (lane >> 4);
  if (px + py + pz > type_limit(type, L.n)) return;
  const size_t nslots = (size_t)L.nmacro * L.ntiles * 384;
  const size_t slot = (size_t)wid * 384 + threadIdx.x;
  TempElem e;
  temp_elem(L, mac, type | (px << 3) | (py << 13) | (pz << 23), e);
  double lr[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) lr[v] = lnrho ? lnrho[e.g1[v]] : 0.0;
  double acc[TEMP_SMAT_ENTRIES];
#pragma unroll
  for (int k = 0; k < TEMP_SMAT_ENTRIES; ++k) acc[k] = 0.0;
  for (int q = 0; q < VMASS_NQ; ++q) {
    const double lam[4] = {qr.lam[q][0], qr.lam[q][1], qr.lam[q][2], qr.lam[q][3]};
    double xq[3], W, gL[4][3], N[10], dN[10][3];
    temp_point<BLEND>(e.G, e.xv, e.gl, lam, qr.w[q] * e.detF, xq, W, gL, N, dN);
    const double wm = W * s1;
    const double wk = W * tk * exp(-(lam[0] * lr[0] + lam[1] * lr[1] + lam[2] * lr[2] + lam[3] * lr[3]));
    int k = 0;
#pragma unroll
    for (int i = 0; i < 10; ++i)
#pragma unroll
      for (int j = i; j < 10; ++j, ++k)
        acc[k] += wm * N[i] * N[j] + wk * (dN[i][0] * dN[j][0] + dN[i][1] * dN[j][1] + dN[i][2] * dN[j][2]);
  }
#pragma unroll
  for (int k = 0; k < TEMP_SMAT_ENTRIES; ++k) S[(size_t)k * nslots + slot] = acc[k];
}

// y += S x with the stored element matrices (y zero-filled by the caller): the
// brick's P2 values of x are staged in LDS, each lane adds its micro-tet's
// product into an LDS box of the brick's nodes, and the box is written out
// (plain stores for nodes inside both the brick and the macro, atomic adds
// for the others).
// Four workgroups per CU asked of the compiler (at most 80 VGPRs, six waves
// per SIMD): the kernel waits on memory latency, so resident waves pay more
// than the extra loads in flight per wave that more registers would allow.
__global__ __launch_bounds__(384, 4) void k_temp_sapply(LevelDev L, const double* __restrict__ S,
                                                     const double* __restrict__ x, double* __restrict__ y) {
  __shared__ double sx[NB2], sy[NB2];
  const int wid = xcd_item(blockIdx.x, gridDim.x);
  const int tile = wid % L.ntiles;
  const int mac = wid / L.ntiles;
  const int ox = L.tiles[3 * tile], oy = L.tiles[3 * tile + 1], oz = L.tiles[3 * tile + 2];
  const int n = L.n, m2 = 2 * n;
  const uint32_t* l2 = L.l2g2 + (size_t)mac * L.nloc2;
  for (int i = threadIdx.x; i < NB2; i += blockDim.x) {
    const int I = 2 * ox + i % B2, J = 2 * oy + (i / B2) % B2, K = 2 * oz + i / (B2 * B2);
    sx[i] = (I + J + K <= m2) ? x[l2[lloc(I, J, K, m2)]] : 0.0;
    sy[i] = 0.0;
  }
  __syncthreads();
  const int type = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int cx = lane & 3, cy = (lane >> 2) & 3, cz = lane >> 4;
  if (ox + cx + oy + cy + oz + cz <= type_limit(type, n)) {
    const size_t nslots = (size_t)L.nmacro * L.ntiles * 384;
    const size_t slot = (size_t)wid * 384 + threadIdx.x;
    ElemIdx e;
    elem_indices(type, cx, cy, cz, e);
    double xs[10], acc[10];
#pragma unroll
    for (int a = 0; a < 10; ++a) {
      xs[a] = sx[e.n2i[a]];
      acc[a] = 0.0;
    }
    int k = 0;
#pragma unroll
    for (int i = 0; i < 10; ++i)
#pragma unroll
      for (int j = i; j < 10; ++j, ++k) {
        const double sij = S[(size_t)k * nslots + slot];
        acc[i] += sij * xs[j];
        if (j != i) acc[j] += sij * xs[i];
      }
#pragma unroll
    for (int a = 0; a < 10; ++a) ldsadd(sy + e.n2i[a], acc[a]);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < NB2; i += blockDim.x) {
    const int lx = i % B2, ly = (i / B2) % B2, lz = i / (B2 * B2);
    const int I = 2 * ox + lx, J = 2 * oy + ly, K = 2 * oz + lz;
    if (I + J + K > m2) continue;
    const size_t g = l2[lloc(I, J, K, m2)];
    const bool excl = wmask(I, J, K, m2) == 15 && lx > 0 && lx < B2 - 1 && ly > 0 && ly < B2 - 1 && lz > 0 && lz < B2 - 1;
    if (excl) y[g] = sy[i];
    else gadd(y + g, sy[i]);
  }
}

// ---- point location and the method of characteristics (Sec. 3) ------------------
struct PointLoc {
  int mac, type, cx, cy, cz;
  double lam[4];
};

__device__ __forceinline__ double min4(const double l[4]) { return fmin(fmin(l[0], l[1]), fmin(l[2], l[3])); }
__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// barycentric coordinates (1 - a - b - c, a, b, c) of the reference point xt in macro mac
__device__ __forceinline__ void macro_bary(const LevelDev& L, const LocDev& loc, int mac, const double xt[3],
                                           double lam[4]) {
  const double* G = L.geo + (size_t)mac * 16;
  const double* Mi = loc.minv + (size_t)mac * 9;
  const double r0 = xt[0] - G[0], r1 = xt[1] - G[1], r2 = xt[2] - G[2];
#pragma unroll
  for (int k = 0; k < 3; ++k) lam[k + 1] = Mi[3 * k] * r0 + Mi[3 * k + 1] * r1 + Mi[3 * k + 2] * r2;
  lam[0] = 1.0 - lam[1] - lam[2] - lam[3];
}

// X: a physical point inside the domain (after clamping)
__device__ void locate_point(const LevelDev& L, const LocDev& loc, const double X[3], PointLoc& o) {
  double best = -1e300;
  int bm = 0;
  double bl[4] = {1.0, 0.0, 0.0, 0.0};
  if (loc.kind == 1) {
    const double r = sqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
    const double d[3] = {X[0] / r, X[1] / r, X[2] / r};
    int bf = 0;
    double bc[3] = {1.0, 1.0, 1.0}, bmin = -1e300;
    for (int f = 0; f < 20; ++f) {
      const double* M = loc.fmat[f];
      const double c0 = M[0] * d[0] + M[1] * d[1] + M[2] * d[2];
      const double c1 = M[3] * d[0] + M[4] * d[1] + M[5] * d[2];
      const double c2 = M[6] * d[0] + M[7] * d[1] + M[8] * d[2];
      const double mn = fmin(c0, fmin(c1, c2));
      if (mn > bmin) {
        bmin = mn;
        bf = f;
        bc[0] = c0;
        bc[1] = c1;
        bc[2] = c2;
      }
    }
    const int nt = loc.n_tan;
    const double cs = bc[0] + bc[1] + bc[2];
    const double xa = nt * bc[0] / cs, xb = nt * bc[1] / cs;
    const int i = clampi((int)floor(fmin(fmax(xa, 0.0), (double)nt)), 0, nt - 1);
    const int j = clampi((int)floor(fmin(fmax(xb, 0.0), (double)nt)), 0, nt - 1 - i);
    const int down = ((xa - i) + (xb - j) > 1.0) && (i + j <= nt - 2);
    const int tri = 2 * (i * nt + j) + down;
    const double t = (r - loc.r_in) / (loc.r_out - loc.r_in) * loc.n_rad;
    const int k = clampi((int)floor(fmin(fmax(t, 0.0), (double)loc.n_rad)), 0, loc.n_rad - 1);
    const int* cand = loc.prism + (((size_t)bf * 2 * nt * nt + tri) * loc.n_rad + k) * 3;
    for (int s = 0; s < 3; ++s) {
      const int m = cand[s];
      const double* G = L.geo + (size_t)m * 16;
      const double gd = G[12] * d[0] + G[13] * d[1] + G[14] * d[2];
      const double rt = (r - G[15]) / gd;
      if (!(rt > 0.0)) continue;
      const double xt[3] = {rt * d[0], rt * d[1], rt * d[2]};
      double lam[4];
      macro_bary(L, loc, m, xt, lam);
      const double mn = min4(lam);
      if (mn > best) {
        best = mn;
        bm = m;
#pragma unroll
        for (int v = 0; v < 4; ++v) bl[v] = lam[v];
      }
    }
  } else {
    for (int m = 0; m < L.nmacro; ++m) {
      double lam[4];
      macro_bary(L, loc, m, X, lam);
      const double mn = min4(lam);
      if (mn > best) {
        best = mn;
        bm = m;
#pragma unroll
        for (int v = 0; v < 4; ++v) bl[v] = lam[v];
      }
    }
  }
  // lattice cube and micro-tet type inside the macro (P1 lattice coordinates)
  const int n = L.n;
  double p[3];
  int c[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    p[k] = fmin(fmax(n * bl[k + 1], 0.0), (double)n);
    c[k] = clampi((int)floor(p[k]), 0, n - 1);
  }
  // a point on the macro's far face may floor to a cube beyond it
  while (c[0] + c[1] + c[2] > n - 1) {
    const int k = (c[0] >= c[1] && c[0] >= c[2]) ? 0 : (c[1] >= c[2] ? 1 : 2);
    --c[k];
  }
  const int sc = c[0] + c[1] + c[2];
  double bt = -1e300;
  o.mac = bm;
  o.type = 0;
  o.cx = c[0];
  o.cy = c[1];
  o.cz = c[2];
  o.lam[0] = 1.0;
  o.lam[1] = o.lam[2] = o.lam[3] = 0.0;
  for (int ty = 0; ty < 6; ++ty) {
    if (sc > type_limit(ty, n)) continue;
    const double r0 = p[0] - c[0] - c_toff[ty][0][0], r1 = p[1] - c[1] - c_toff[ty][0][1],
                 r2 = p[2] - c[2] - c_toff[ty][0][2];
    const double* T = loc.tinv6[ty];
    double lam[4];
#pragma unroll
    for (int k = 0; k < 3; ++k) lam[k + 1] = T[3 * k] * r0 + T[3 * k + 1] * r1 + T[3 * k + 2] * r2;
    lam[0] = 1.0 - lam[1] - lam[2] - lam[3];
    const double mn = min4(lam);
    if (mn > bt) {
      bt = mn;
      o.type = ty;
#pragma unroll
      for (int v = 0; v < 4; ++v) o.lam[v] = lam[v];
    }
  }
}

// global P2 nodes and basis values of a located point
__device__ __forceinline__ void point_basis(const LevelDev& L, const PointLoc& o, size_t g2[10], double N[10]) {
  const int m2 = 2 * L.n;
  const uint32_t* l2 = L.l2g2 + (size_t)o.mac * L.nloc2;
  int I2[10], J2[10], K2[10];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    I2[v] = 2 * (o.cx + c_toff[o.type][v][0]);
    J2[v] = 2 * (o.cy + c_toff[o.type][v][1]);
    K2[v] = 2 * (o.cz + c_toff[o.type][v][2]);
    N[v] = o.lam[v] * (2.0 * o.lam[v] - 1.0);
  }
#pragma unroll
  for (int ed = 0; ed < 6; ++ed) {
    const int i = EV0(ed), j = EV1(ed);
    I2[4 + ed] = (I2[i] + I2[j]) >> 1;
    J2[4 + ed] = (J2[i] + J2[j]) >> 1;
    K2[4 + ed] = (K2[i] + K2[j]) >> 1;
    N[4 + ed] = 4.0 * o.lam[i] * o.lam[j];
  }
#pragma unroll
  for (int a = 0; a < 10; ++a) g2[a] = l2[lloc(I2[a], J2[a], K2[a], m2)];
}

// move a point that left the domain back onto it
__device__ __forceinline__ void clamp_to_domain(const LocDev& loc, double X[3]) {
  if (loc.kind == 1) {
    const double r = sqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
    const double rc = fmin(fmax(r, loc.r_in), loc.r_out);
    if (rc != r) {
      const double f = rc / r;
      X[0] *= f;
      X[1] *= f;
      X[2] *= f;
    }
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) X[k] = fmin(fmax(X[k], 0.0), 1.0);
  }
}

// velocity at X (clamped first) and time t - tau + theta tau
__device__ __forceinline__ void mmoc_vel(const LevelDev& L, const LocDev& loc, const double* __restrict__ un,
                                         const double* __restrict__ uo, double theta, double X[3], double v[3]) {
  clamp_to_domain(loc, X);
  PointLoc o;
  locate_point(L, loc, X, o);
  size_t g2[10];
  double N[10];
  point_basis(L, o, g2, N);
  const size_t N2 = (size_t)L.n2;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < 10; ++a) s += N[a] * (theta * un[g2[a] + c * N2] + (1.0 - theta) * uo[g2[a] + c * N2]);
    v[c] = s;
  }
}

// One thread per (macro, P2 lattice point); the macro owning the node writes it.
__global__ __launch_bounds__(256) void k_mmoc(LevelDev L, LocDev loc, const double* __restrict__ F,
                                              const double* __restrict__ un, const double* __restrict__ uo, double tau,
                                              double* __restrict__ out) {
  const long long gid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int m2 = 2 * L.n, nl = L.nloc2;
  if (gid >= (long long)nl * L.nmacro) return;
  const int mac = (int)(gid / nl);
  const int t = (int)(gid - (long long)mac * nl);
  int I, J, K;
  lattice_of(t, m2, I, J, K);
  if (!L.own[(size_t)mac * 16 + wmask(I, J, K, m2)]) return;
  const size_t g = L.l2g2[(size_t)mac * nl + t];
  const double* G = L.geo + (size_t)mac * 16;
  double X0[3];
  lattice_x<double>(G, I, J, K, m2, X0);
  if (L.blend) {
    const double s = G[12] * X0[0] + G[13] * X0[1] + G[14] * X0[2] + G[15];
    const double f = s / sqrt(X0[0] * X0[0] + X0[1] * X0[1] + X0[2] * X0[2]);
    X0[0] *= f;
    X0[1] *= f;
    X0[2] *= f;
  }
  const size_t N2 = (size_t)L.n2;
  // classical Runge-Kutta backwards: stage velocities at t, t - tau/2 (twice), t - tau
  const double k1[3] = {un[g], un[g + N2], un[g + 2 * N2]};
  double P[3], k2[3], k3[3], k4[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) P[c] = X0[c] - 0.5 * tau * k1[c];
  mmoc_vel(L, loc, un, uo, 0.5, P, k2);
#pragma unroll
  for (int c = 0; c < 3; ++c) P[c] = X0[c] - 0.5 * tau * k2[c];
  mmoc_vel(L, loc, un, uo, 0.5, P, k3);
#pragma unroll
  for (int c = 0; c < 3; ++c) P[c] = X0[c] - tau * k3[c];
  mmoc_vel(L, loc, un, uo, 0.0, P, k4);
#pragma unroll
  for (int c = 0; c < 3; ++c) P[c] = X0[c] - tau / 6.0 * (k1[c] + 2.0 * k2[c] + 2.0 * k3[c] + k4[c]);
  clamp_to_domain(loc, P);
  PointLoc o;
  locate_point(L, loc, P, o);
  size_t g2[10];
  double N[10];
  point_basis(L, o, g2, N);
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < 10; ++a) s += N[a] * F[g2[a]];
  out[g] = s;
}

__global__ void k_scalar_dirichlet(const uint32_t* __restrict__ node, const uint8_t* __restrict__ kind, int nb,
                                   double* v, int set, double vin, double vout) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  v[node[i]] = set ? (kind[i] == 2 ? vout : vin) : 0.0;
}

// ---- diag(A) (no free-slip projection, Sec. 5.2.2) ---------------------------
template <typename R, bool BLEND>
__global__ __launch_bounds__(384) void k_diag(LevelDev L, const R* __restrict__ eta, R* __restrict__ dout) {
  __shared__ R sy[3 * NB2];
  __shared__ R seta[NB1];
  const int wid = xcd_item(blockIdx.x, gridDim.x);
  const int tile = wid % L.ntiles;
  const int mac = wid / L.ntiles;
  const int ox = L.tiles[3 * tile], oy = L.tiles[3 * tile + 1], oz = L.tiles[3 * tile + 2];
  const int n = L.n, m2 = 2 * L.n;
  const uint32_t* l2 = L.l2g2 + (size_t)mac * L.nloc2;
  const uint32_t* l1 = L.l2g1 + (size_t)mac * L.nloc1;
  const R* G = geo_of<R>(L) + (size_t)mac * 16;
  const size_t N2 = (size_t)L.n2;
  for (int i = threadIdx.x; i < 3 * NB2; i += blockDim.x) sy[i] = 0;
  for (int i = threadIdx.x; i < NB1; i += blockDim.x) {
    const int I = ox + i % B1, J = oy + (i / B1) % B1, K = oz + i / (B1 * B1);
    seta[i] = (I + J + K <= n) ? eta[l1[lloc(I, J, K, n)]] : R(0);
  }
  __syncthreads();
  const int type = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int cx = lane & 3, cy = (lane >> 2) & 3, cz = lane >> 4;
  const int px = ox + cx, py = oy + cy, pz = oz + cz;
  if (px + py + pz <= type_limit(type, n)) {
    ElemIdx e;
    elem_indices(type, cx, cy, cz, e);
    const R* TI = tinv_of<R>(L) + ((size_t)mac * 6 + type) * 10;
    R gl[4][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      gl[1][k] = TI[k];
      gl[2][k] = TI[3 + k];
      gl[3][k] = TI[6 + k];
      gl[0][k] = -(gl[1][k] + gl[2][k] + gl[3][k]);
    }
    const R wdetF = R(QW) * TI[9];
    R xv[4][3], xs[3] = {0, 0, 0};
    if (BLEND) {
      elem_vertices<R>(G, type, px, py, pz, n, xv);
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int k = 0; k < 3; ++k) xs[k] += xv[v][k];
    }
    R et[4], set = 0;
#pragma unroll
    for (int v = 0; v < 4; ++v) { et[v] = seta[e.n1i[v]]; set += et[v]; }
    R D[3][10];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int a = 0; a < 10; ++a) D[c][a] = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      R xq[3];
      if (BLEND) {
#pragma unroll
        for (int k = 0; k < 3; ++k) xq[k] = R(QB) * xs[k] + R(QA - QB) * xv[q][k];
      }
      QGeo<R, BLEND> geo;
      geo.eval(G, xq, wdetF);
      const R we = geo.W * (R(QB) * set + R(QA - QB) * et[q]);
#pragma unroll
      for (int a = 0; a < 10; ++a) {
        R gN[3];
        if (a < 4) {
          const R f = (a == q) ? R(4.0 * QA - 1.0) : R(C1);
#pragma unroll
          for (int k = 0; k < 3; ++k) gN[k] = f * gl[a][k];
        } else {
          const int i = EV0(a - 4), j = EV1(a - 4);
          const R li = (i == q) ? R(4.0 * QA) : R(4.0 * QB), lj = (j == q) ? R(4.0 * QA) : R(4.0 * QB);
#pragma unroll
          for (int k = 0; k < 3; ++k) gN[k] = lj * gl[i][k] + li * gl[j][k];
        }
        geo.JinvT(gN);
        const R g2 = gN[0] * gN[0] + gN[1] * gN[1] + gN[2] * gN[2];
#pragma unroll
        for (int c = 0; c < 3; ++c) D[c][a] += we * (g2 + gN[c] * gN[c] * R(1.0 / 3.0));
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int a = 0; a < 10; ++a) ldsadd(sy + c * NB2 + e.n2i[a], D[c][a]);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < NB2; i += blockDim.x) {
    const int lx = i % B2, ly = (i / B2) % B2, lz = i / (B2 * B2);
    const int I = 2 * ox + lx, J = 2 * oy + ly, K = 2 * oz + lz;
    if (I + J + K > m2) continue;
    const size_t g = l2[lloc(I, J, K, m2)];
    const bool excl = wmask(I, J, K, m2) == 15 && lx > 0 && lx < B2 - 1 && ly > 0 && ly < B2 - 1 && lz > 0 && lz < B2 - 1;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (excl) dout[g + c * N2] = sy[c * NB2 + i];
      else gadd(dout + g + c * N2, sy[c * NB2 + i]);
    }
  }
}

// ---- P1 mass with weight 1/eta (Schur approximation M_{1/eta}) --------------
// DIAG: the diagonal of the same matrix (p unused)
template <typename R, bool BLEND, bool DIAG>
__global__ __launch_bounds__(384) void k_mass(LevelDev L, const R* __restrict__ eta, const R* __restrict__ p,
                                              R* __restrict__ y) {
  __shared__ R seta[NB1], sp[NB1], sy[NB1];
  const int wid = xcd_item(blockIdx.x, gridDim.x);
  const int tile = wid % L.ntiles;
  const int mac = wid / L.ntiles;
  const int ox = L.tiles[3 * tile], oy = L.tiles[3 * tile + 1], oz = L.tiles[3 * tile + 2];
  const int n = L.n;
  const uint32_t* l1 = L.l2g1 + (size_t)mac * L.nloc1;
  const R* G = geo_of<R>(L) + (size_t)mac * 16;
  for (int i = threadIdx.x; i < NB1; i += blockDim.x) {
    const int I = ox + i % B1, J = oy + (i / B1) % B1, K = oz + i / (B1 * B1);
    const bool in = I + J + K <= n;
    const size_t g = in ? l1[lloc(I, J, K, n)] : 0;
    seta[i] = in ? eta[g] : R(1);
    sp[i] = (in && !DIAG) ? p[g] : R(0);
    sy[i] = 0;
  }
  __syncthreads();
  const int type = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int cx = lane & 3, cy = (lane >> 2) & 3, cz = lane >> 4;
  const int px = ox + cx, py = oy + cy, pz = oz + cz;
  if (px + py + pz <= type_limit(type, n)) {
    ElemIdx e;
    elem_indices(type, cx, cy, cz, e);
    const R* TI = tinv_of<R>(L) + ((size_t)mac * 6 + type) * 10;
    const R wdetF = R(QW) * TI[9];
    R xv[4][3], xs[3] = {0, 0, 0};
    if (BLEND) {
      elem_vertices<R>(G, type, px, py, pz, n, xv);
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int k = 0; k < 3; ++k) xs[k] += xv[v][k];
    }
    R et[4], pp[4], set = 0, spp = 0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      et[v] = seta[e.n1i[v]];
      pp[v] = sp[e.n1i[v]];
      set += et[v];
      spp += pp[v];
    }
    R SM = 0, DM[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      R xq[3];
      if (BLEND) {
#pragma unroll
        for (int k = 0; k < 3; ++k) xq[k] = R(QB) * xs[k] + R(QA - QB) * xv[q][k];
      }
      QGeo<R, BLEND> geo;
      geo.eval(G, xq, wdetF);
      const R etaq = R(QB) * set + R(QA - QB) * et[q];
      const R v = DIAG ? geo.W / etaq : geo.W * (R(QB) * spp + R(QA - QB) * pp[q]) / etaq;
      SM += v;
      DM[q] = v;
    }
    if (DIAG) {
      // sum_q w_q lambda_i(q)^2 with lambda_i(q) = QB + (QA - QB) delta_iq
#pragma unroll
      for (int i = 0; i < 4; ++i) ldsadd(sy + e.n1i[i], R(QB * QB) * SM + R(QA * QA - QB * QB) * DM[i]);
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) ldsadd(sy + e.n1i[i], R(QB) * SM + R(QA - QB) * DM[i]);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < NB1; i += blockDim.x) {
    const int lx = i % B1, ly = (i / B1) % B1, lz = i / (B1 * B1);
    const int I = ox + lx, J = oy + ly, K = oz + lz;
    if (I + J + K > n) continue;
    const size_t g = l1[lloc(I, J, K, n)];
    const bool excl = wmask(I, J, K, n) == 15 && lx > 0 && lx < B1 - 1 && ly > 0 && ly < B1 - 1 && lz > 0 && lz < B1 - 1;
    if (excl) y[g] = sy[i];
    else gadd(y + g, sy[i]);
  }
}

// ---- buoyancy right-hand side f = int scale T_h r_hat . phi (FP64) ------------
// ---- and adjoint gradient g_m, g_T (FP64) -------------------------------------
// MODE 0: rhs (input T (P2 scalar) -> f (P2 vector))
// MODE 1: gradient (inputs u, lam (P2 vectors), eta -> gm (P1), gT (P2 scalar))
template <bool BLEND, int MODE>
__global__ __launch_bounds__(384) void k_rhs_grad(LevelDev L, const double* __restrict__ T,
                                                  const double* __restrict__ u, const double* __restrict__ lam,
                                                  const double* __restrict__ eta, double* __restrict__ out2,
                                                  double* __restrict__ out1, double scale) {
  constexpr int NIN = MODE == 0 ? 1 : 6;
  constexpr int NOUT = MODE == 0 ? 3 : 1;
  __shared__ double sx[NIN * NB2];
  __shared__ double sy[NOUT * NB2];
  __shared__ double seta[MODE == 1 ? NB1 : 1], sg[MODE == 1 ? NB1 : 1];
  const int wid = xcd_item(blockIdx.x, gridDim.x);
  const int tile = wid % L.ntiles;
  const int mac = wid / L.ntiles;
  const int ox = L.tiles[3 * tile], oy = L.tiles[3 * tile + 1], oz = L.tiles[3 * tile + 2];
  const int n = L.n, m2 = 2 * L.n;
  const uint32_t* l2 = L.l2g2 + (size_t)mac * L.nloc2;
  const uint32_t* l1 = L.l2g1 + (size_t)mac * L.nloc1;
  const double* G = L.geo + (size_t)mac * 16;
  const uint8_t* bact = L.bact + (size_t)mac * 16;
  const size_t N2 = (size_t)L.n2;
  for (int i = threadIdx.x; i < NB2; i += blockDim.x) {
    const int lx = i % B2, ly = (i / B2) % B2, lz = i / (B2 * B2);
    const int I = 2 * ox + lx, J = 2 * oy + ly, K = 2 * oz + lz;
    const bool in = I + J + K <= m2;
    const size_t g = in ? l2[lloc(I, J, K, m2)] : 0;
    if (MODE == 0) {
      sx[i] = in ? T[g] : 0.0;
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        sx[c * NB2 + i] = in ? u[g + c * N2] : 0.0;
        sx[(3 + c) * NB2 + i] = in ? lam[g + c * N2] : 0.0;
      }
    }
#pragma unroll
    for (int c = 0; c < NOUT; ++c) sy[c * NB2 + i] = 0;
  }
  if (MODE == 1) {
    for (int i = threadIdx.x; i < NB1; i += blockDim.x) {
      const int I = ox + i % B1, J = oy + (i / B1) % B1, K = oz + i / (B1 * B1);
      seta[i] = (I + J + K <= n) ? eta[l1[lloc(I, J, K, n)]] : 0.0;
      sg[i] = 0;
    }
  }
  __syncthreads();
  const int type = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int cx = lane & 3, cy = (lane >> 2) & 3, cz = lane >> 4;
  const int px = ox + cx, py = oy + cy, pz = oz + cz;
  if (px + py + pz <= type_limit(type, n)) {
    ElemIdx e;
    elem_indices(type, cx, cy, cz, e);
    const double* TI = L.tinv + ((size_t)mac * 6 + type) * 10;
    double gl[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int k = 0; k < 3; ++k) gl[r][k] = TI[3 * r + k];
    const double wdetF = QW * TI[9];
    double xv[4][3], xs[3] = {0, 0, 0};
    elem_vertices<double>(G, type, px, py, pz, n, xv);
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int k = 0; k < 3; ++k) xs[k] += xv[v][k];
    double SV[3] = {0, 0, 0}, VQ[3][4];
    double SG = 0, DG[4];
    double Uv[6][10];
#pragma unroll
    for (int c = 0; c < NIN; ++c)
#pragma unroll
      for (int a = 0; a < 10; ++a) Uv[c][a] = sx[c * NB2 + e.n2i[a]];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double xq[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) xq[k] = QB * xs[k] + (QA - QB) * xv[q][k];
      QGeo<double, BLEND> geo;
      geo.eval(G, xq, wdetF);
      double dir[3];
      {
        double ri = 1.0 / sqrt(xq[0] * xq[0] + xq[1] * xq[1] + xq[2] * xq[2]);
        dir[0] = xq[0] * ri;
        dir[1] = xq[1] * ri;
        dir[2] = xq[2] * ri;
      }
      // value of a P2 field at qp q
      auto val_at = [&](const double* f) {
        double sv = f[0] + f[1] + f[2] + f[3];
        double se = f[4] + f[5] + f[6] + f[7] + f[8] + f[9];
        double eq = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (i != q) eq += f[eidx(i, q)];
        return NV_OTH * sv + (NV_OWN - NV_OTH) * f[q] + NE_OTH * se + (NE_OWN - NE_OTH) * eq;
      };
      if (MODE == 0) {
        const double Tq = val_at(Uv[0]);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          double v = scale * geo.W * Tq * dir[c];
          SV[c] += v;
          VQ[c][q] = v;
        }
      } else {
        double Gu[3][3], Gl[3][3];
#pragma unroll
        for (int f = 0; f < 2; ++f) {
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const double* Uc = Uv[3 * f + c];
            double g4[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              double s = 0;
#pragma unroll
              for (int j = 0; j < 4; ++j)
                if (j != i) s += Uc[eidx(i, j)];
              g4[i] = C1 * Uc[i] + 4.0 * QB * s + KAP * (i == q ? Uc[i] : Uc[eidx(i, q)]);
            }
            double* Gr = f == 0 ? Gu[c] : Gl[c];
#pragma unroll
            for (int k = 0; k < 3; ++k)
              Gr[k] = (g4[1] - g4[0]) * gl[0][k] + (g4[2] - g4[0]) * gl[1][k] + (g4[3] - g4[0]) * gl[2][k];
            geo.rowJinv(Gr);
          }
        }
        double dd = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int k = 0; k < 3; ++k) dd += 0.25 * (Gu[c][k] + Gu[k][c]) * (Gl[c][k] + Gl[k][c]);
        dd -= (Gu[0][0] + Gu[1][1] + Gu[2][2]) * (Gl[0][0] + Gl[1][1] + Gl[2][2]) / 3.0;
        SG += geo.W * dd;
        DG[q] = geo.W * dd;
        double lr = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) lr += val_at(Uv[3 + c]) * dir[c];
        const double v = scale * geo.W * lr;
        SV[0] += v;
        VQ[0][q] = v;
      }
    }
#pragma unroll
    for (int c = 0; c < NOUT; ++c) {
      double* yc = sy + c * NB2;
#pragma unroll
      for (int i = 0; i < 4; ++i) ldsadd(yc + e.n2i[i], NV_OTH * SV[c] + (NV_OWN - NV_OTH) * VQ[c][i]);
#pragma unroll
      for (int ed = 0; ed < 6; ++ed) {
        const int i = EV0(ed), j = EV1(ed);
        ldsadd(yc + e.n2i[4 + ed], NE_OTH * SV[c] + (NE_OWN - NE_OTH) * (VQ[c][i] + VQ[c][j]));
      }
    }
    if (MODE == 1) {
      double et[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) et[v] = seta[e.n1i[v]];
#pragma unroll
      for (int i = 0; i < 4; ++i) ldsadd(sg + e.n1i[i], -2.0 * et[i] * (QB * SG + (QA - QB) * DG[i]));
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < NB2; i += blockDim.x) {
    const int lx = i % B2, ly = (i / B2) % B2, lz = i / (B2 * B2);
    const int I = 2 * ox + lx, J = 2 * oy + ly, K = 2 * oz + lz;
    if (I + J + K > m2) continue;
    const size_t g = l2[lloc(I, J, K, m2)];
    const bool excl = wmask(I, J, K, m2) == 15 && lx > 0 && lx < B2 - 1 && ly > 0 && ly < B2 - 1 && lz > 0 && lz < B2 - 1;
#pragma unroll
    for (int c = 0; c < NOUT; ++c) {
      if (excl) out2[g + c * N2] = sy[c * NB2 + i];
      else gadd(out2 + g + c * N2, sy[c * NB2 + i]);
    }
  }
  if (MODE == 1) {
    for (int i = threadIdx.x; i < NB1; i += blockDim.x) {
      const int lx = i % B1, ly = (i / B1) % B1, lz = i / (B1 * B1);
      const int I = ox + lx, J = oy + ly, K = oz + lz;
      if (I + J + K > n) continue;
      const size_t g = l1[lloc(I, J, K, n)];
      const bool excl = wmask(I, J, K, n) == 15 && lx > 0 && lx < B1 - 1 && ly > 0 && ly < B1 - 1 && lz > 0 && lz < B1 - 1;
      if (excl) out1[g] = sg[i];
      else gadd(out1 + g, sg[i]);
    }
  }
  (void)bact;
}

// ---- grid transfers ------------------------------------------------------------
// Nested P2 spaces: the fine P2 lattice of a macro (side 4 nc) contains the
// coarse one (side 2 nc).  Fine point J lies in the coarse cube
// p_k = (J_k - 1) div 4 (J_k > 0; else 0) at local position f = J - 4p in
// quarter units; its coarse micro-tet is "up" for |f| <= 4, one of the four
// octahedron tets for 4 < |f| <= 8 (first one containing it), "down" above.
// Prolongation evaluates the coarse P2 basis there (weights are multiples of
// 1/8, tabulated per level on the host); restriction is the transpose.  Each
// fine node is handled by the brick of its coarse cube in its owning macro
// only.
// MODE 0: out = P in;  1: out = P^T in;  2: out += P in;  3: out = P^T (in - in2).
// One workgroup per (macro, coarse brick): the brick's coarse P2 values are
// staged in LDS (prolongation) or accumulated there in FP64 (restriction);
// the fine points of the brick and their nonzero coarse weights come from the
// level's transfer table.
template <typename R, int MODE>
__global__ __launch_bounds__(256) void k_transfer(LevelDev Lc, LevelDev Lf, const R* __restrict__ in,
                                                  const R* __restrict__ in2, R* __restrict__ out, int bcmode) {
  constexpr bool PRO = MODE == 0 || MODE == 2;
  constexpr int NB = 4;   // fine points per thread and batch (all loads of a batch in flight together)
  __shared__ double sc[3 * NB2];   // FP64 staging / accumulation (fast LDS atomics)
  const int wid = xcd_item(blockIdx.x, gridDim.x);
  const int tile = wid % Lc.ntiles;
  const int mac = wid / Lc.ntiles;
  const int ox = Lc.tiles[3 * tile], oy = Lc.tiles[3 * tile + 1], oz = Lc.tiles[3 * tile + 2];
  const int nc = Lc.n, mc2 = 2 * nc, mf2 = 4 * nc;
  const uint32_t* l2c = Lc.l2g2 + (size_t)mac * Lc.nloc2;
  const uint32_t* l2f = Lf.l2g2 + (size_t)mac * Lf.nloc2;
  const R* G = geo_of<R>(Lc) + (size_t)mac * 16;
  const uint8_t* bact = Lc.bact + (size_t)mac * 16;
  // the macro's 16 ownership bytes (16-byte aligned), held in registers
  const uint4 ownw = *reinterpret_cast<const uint4*>(Lf.own + (size_t)mac * 16);
  const size_t Nc = (size_t)Lc.n2, Nf = (size_t)Lf.n2;
  {
    // coarse brick: staged values (prolongation) or zeroed accumulators
    constexpr int NS = (NB2 + 255) / 256;
    size_t g[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const int i = threadIdx.x + 256 * k;
      const int lx = i % B2, ly = (i / B2) % B2, lz = i / (B2 * B2);
      const int I = 2 * ox + lx, J = 2 * oy + ly, K = 2 * oz + lz;
      g[k] = (PRO && i < NB2 && I + J + K <= mc2) ? p2_gidx(l2c, mac, I, J, K, mc2, wmask(I, J, K, mc2))
                                                   : ~(size_t)0;
    }
    R v[NS][3];
#pragma unroll
    for (int k = 0; k < NS; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) v[k][c] = g[k] != ~(size_t)0 ? in[g[k] + c * Nc] : R(0);
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const int i = threadIdx.x + 256 * k;
      if (i < NB2) {
        sc[i] = v[k][0];
        sc[NB2 + i] = v[k][1];
        sc[2 * NB2 + i] = v[k][2];
      }
    }
  }
  __syncthreads();
  const int e0 = Lc.xoff[tile], e1 = Lc.xoff[tile + 1];
  for (int base = e0; base < e1; base += NB * 256) {
    int4 ta[NB], tb[NB];
    bool ok[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const int e = base + k * 256 + threadIdx.x;
      ok[k] = e < e1;
      if (ok[k]) {
        ta[k] = Lc.xtab[2 * e];
        tb[k] = Lc.xtab[2 * e + 1];
      } else {
        ta[k] = make_int4(0, 0, 0, 0);
        tb[k] = ta[k];
      }
    }
    size_t gf[NB];
    int mask[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const int JX = ta[k].x & 1023, JY = (ta[k].x >> 10) & 1023, JZ = (ta[k].x >> 20) & 1023;
      mask[k] = wmask(JX, JY, JZ, mf2);
      const int mk = mask[k];
      const unsigned ow = mk < 4 ? ownw.x : (mk < 8 ? ownw.y : (mk < 12 ? ownw.z : ownw.w));
      ok[k] = ok[k] && ((ow >> (8 * (mk & 3))) & 0xffu) != 0;
      gf[k] = ok[k] ? p2_gidx(l2f, mac, JX, JY, JZ, mf2, mk) : 0;
    }
    R v[NB][3];
    if (!PRO || MODE == 2) {
#pragma unroll
      for (int k = 0; k < NB; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) v[k][c] = ok[k] ? (MODE == 2 ? out : in)[gf[k] + c * Nf] : R(0);
      if (MODE == 3) {
#pragma unroll
        for (int k = 0; k < NB; ++k)
#pragma unroll
          for (int c = 0; c < 3; ++c) v[k][c] -= ok[k] ? in2[gf[k] + c * Nf] : R(0);
      }
    }
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      if (!ok[k]) continue;
      const int JX = ta[k].x & 1023, JY = (ta[k].x >> 10) & 1023, JZ = (ta[k].x >> 20) & 1023;
      const int nnz = ta[k].y;
      const unsigned wd[5] = {(unsigned)ta[k].z, (unsigned)ta[k].w, (unsigned)tb[k].x, (unsigned)tb[k].y,
                              (unsigned)tb[k].z};
      if (PRO) {
        R w3[3] = {0, 0, 0};
#pragma unroll
        for (int j = 0; j < 10; ++j) {
          if (j < nnz) {
            const unsigned f = (wd[j >> 1] >> (16 * (j & 1))) & 0x3fffu;
            const int idx = (int)(f & 1023u), w = (int)(f >> 10) - 1;
#pragma unroll
            for (int c = 0; c < 3; ++c) w3[c] += R(w) * R(sc[c * NB2 + idx]);
          }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) w3[c] *= R(0.125);
        if (bcmode & BCM_OUT) {
          // fine node class = coarse sub-simplex class (same macro, nested)
          const int act = Lf.bact[(size_t)mac * 16 + mask[k]];
          bc_project<R>(act, G, JX, JY, JZ, mf2, w3[0], w3[1], w3[2]);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) out[gf[k] + c * Nf] = (MODE == 2 ? v[k][c] : R(0)) + w3[c];
      } else {
        if (bcmode & BCM_IN)
          bc_project<R>(Lf.bact[(size_t)mac * 16 + mask[k]], G, JX, JY, JZ, mf2, v[k][0], v[k][1], v[k][2]);
#pragma unroll
        for (int j = 0; j < 10; ++j) {
          if (j < nnz) {
            const unsigned f = (wd[j >> 1] >> (16 * (j & 1))) & 0x3fffu;
            const int idx = (int)(f & 1023u);
            const double wf = ((int)(f >> 10) - 1) * 0.125;
            ldsadd(sc + idx, wf * double(v[k][0]));
            ldsadd(sc + NB2 + idx, wf * double(v[k][1]));
            ldsadd(sc + 2 * NB2 + idx, wf * double(v[k][2]));
          }
        }
      }
    }
  }
  if (!PRO) {
    __syncthreads();
    for (int i = threadIdx.x; i < NB2; i += blockDim.x) {
      const int lx = i % B2, ly = (i / B2) % B2, lz = i / (B2 * B2);
      const int I = 2 * ox + lx, J = 2 * oy + ly, K = 2 * oz + lz;
      if (I + J + K > mc2) continue;
      const int mask = wmask(I, J, K, mc2);
      R v0 = R(sc[i]), v1 = R(sc[NB2 + i]), v2 = R(sc[2 * NB2 + i]);
      if (bcmode & BCM_OUT) {
        const int act = bact[mask];
        if (act == ACT_DIR) continue;
        bc_project<R>(act, G, I, J, K, mc2, v0, v1, v2);
      }
      const size_t g = p2_gidx(l2c, mac, I, J, K, mc2, mask);
      const bool excl = mask == 15 && lx > 0 && lx < B2 - 1 && ly > 0 && ly < B2 - 1 && lz > 0 && lz < B2 - 1;
      if (excl) {
        out[g] = v0;
        out[g + Nc] = v1;
        out[g + 2 * Nc] = v2;
      } else {
        gadd(out + g, v0);
        gadd(out + g + Nc, v1);
        gadd(out + g + 2 * Nc, v2);
      }
    }
  }
}

// nodal injection of a P1 field to the next coarser level (coarse node = fine node)
template <typename R>
__global__ void k_inject(LevelDev Lc, LevelDev Lf, const R* __restrict__ vf, R* __restrict__ vc) {
  const int mac = blockIdx.y;
  const int nc = Lc.n;
  for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < Lc.nloc1; l += gridDim.x * blockDim.x) {
    // decode lattice point from local index (K-major, then J, then I)
    int K = 0;
    while (tetc(nc) - tetc(nc - K - 1) <= l) ++K;
    int r = l - (int)(tetc(nc) - tetc(nc - K));
    const int s = nc - K;
    int J = 0;
    while (r >= s - J + 1) { r -= s - J + 1; ++J; }
    const int I = r;
    if (!Lc.own[(size_t)mac * 16 + wmask(I, J, K, nc)]) continue;
    const size_t gc = Lc.l2g1[(size_t)mac * Lc.nloc1 + l];
    const size_t gf = Lf.l2g1[(size_t)mac * Lf.nloc1 + lloc(2 * I, 2 * J, 2 * K, 2 * nc)];
    vc[gc] = vf[gf];
  }
}

// velocity projection over boundary node lists
template <typename R>
__global__ void k_project(BcDev bc, long long n2, R* v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < bc.ndir) {
    const size_t g = bc.dir[i];
    v[g] = 0;
    v[g + n2] = 0;
    v[g + 2 * n2] = 0;
  } else if (i < bc.ndir + bc.nfs) {
    const int k = i - bc.ndir;
    const size_t g = bc.fs[k];
    const double* nr = bc.nrm + 3 * (size_t)k;
    R a = v[g], b = v[g + n2], c = v[g + 2 * n2];
    R dn = a * R(nr[0]) + b * R(nr[1]) + c * R(nr[2]);
    v[g] = a - dn * R(nr[0]);
    v[g + n2] = b - dn * R(nr[1]);
    v[g + 2 * n2] = c - dn * R(nr[2]);
  }
}

// ---- vector kernels --------------------------------------------------------------
template <typename R> __global__ void k_fill(R* x, R a, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) x[i] = a;
}
template <typename R> __global__ void k_copy(const R* __restrict__ x, R* __restrict__ y, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) y[i] = x[i];
}
template <typename R> __global__ void k_axpy(R a, const R* __restrict__ x, R* __restrict__ y, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) y[i] += a * x[i];
}
template <typename R> __global__ void k_axpby(R a, const R* __restrict__ x, R b, R* __restrict__ y, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) y[i] = a * x[i] + b * y[i];
}
template <typename R> __global__ void k_scale(R a, R* x, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) x[i] *= a;
}
template <typename R> __global__ void k_mul(const R* __restrict__ a, const R* __restrict__ x, R* __restrict__ y, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) y[i] = a[i] * x[i];
}
template <typename A, typename B> __global__ void k_convert(const A* __restrict__ x, B* __restrict__ y, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) y[i] = (B)x[i];
}
template <typename R> __global__ void k_invert(const R* __restrict__ d, R* __restrict__ y, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] = d[i] != R(0) ? R(1) / d[i] : R(1);
}
__global__ void k_exp(const double* __restrict__ x, double* __restrict__ y, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) y[i] = exp(x[i]);
}
// Chebyshev smoother pieces (fused vector updates).  xin = 0: x enters as zero
// and is not read.
template <typename R>
__global__ void k_cheb_start(const R* __restrict__ b, const R* __restrict__ t, const R* __restrict__ dinv, R c1,
                             R* __restrict__ r, R* __restrict__ d, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const R ri = t ? b[i] - t[i] : b[i];
    r[i] = ri;
    d[i] = c1 * dinv[i] * ri;
  }
}
template <typename R>
__global__ void k_cheb_one(const R* __restrict__ b, const R* __restrict__ t, const R* __restrict__ dinv, R c1,
                           R* __restrict__ x, int xin, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const R ri = t ? b[i] - t[i] : b[i];
    const R di = c1 * dinv[i] * ri;
    x[i] = xin ? x[i] + di : di;
  }
}
template <typename R>
__global__ void k_cheb_step(const R* __restrict__ t, const R* __restrict__ dinv, R c1, R c2, R* __restrict__ r,
                            R* __restrict__ x, R* __restrict__ d, int xin, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const R ri = r[i] - t[i];
    const R di = d[i];
    r[i] = ri;
    x[i] = xin ? x[i] + di : di;
    d[i] = c1 * dinv[i] * ri + c2 * di;
  }
}
template <typename R>
__global__ void k_cheb_last(const R* __restrict__ t, const R* __restrict__ dinv, R c1, R c2, const R* __restrict__ r,
                            const R* __restrict__ d, R* __restrict__ x, int xin, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const R ri = r[i] - t[i];
    const R di = d[i];
    const R xi = xin ? x[i] + di : di;
    x[i] = xi + (c1 * dinv[i] * ri + c2 * di);
  }
}
template <typename R>
__global__ void k_sub(const R* __restrict__ b, const R* __restrict__ t, R* __restrict__ r, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    r[i] = b[i] - t[i];
}

template <typename R>
__global__ __launch_bounds__(256) void k_dot(const R* __restrict__ x, const R* __restrict__ y, long long n, double* partial) {
  __shared__ double red[256];
  double s = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    s += (double)x[i] * (double)y[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}
// x += a p; r += b q; partial[block] = sum of the new r_i^2 (FP64)
template <typename R>
__global__ __launch_bounds__(256) void k_axpy2_nrm(R a, const R* __restrict__ p, R* __restrict__ x, R b,
                                                   const R* __restrict__ q, R* __restrict__ r, long long n,
                                                   double* partial) {
  __shared__ double red[256];
  double s = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    x[i] += a * p[i];
    const R ri = r[i] + b * q[i];
    r[i] = ri;
    s += (double)ri * (double)ri;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}
__global__ __launch_bounds__(256) void k_sum(const double* __restrict__ partial, int np, double* out) {
  __shared__ double red[256];
  double s = 0;
  for (int i = threadIdx.x; i < np; i += 256) s += partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}


// ---- device-resident Jacobi-preconditioned CG ----------------------------------
// Scalars and partial sums live on the device so that iterations need no host
// round trip.  Partial-sum layout (DOT_BLOCKS = NB): [0, NB) p.q; then for
// parity 0 and 1: [NB + 2 NB k, +NB) r.r and [2 NB + 2 NB k, +NB) r.z.
// Iteration i writes the r.r / r.z partials of parity i & 1 and reads those of
// the other parity as the previous r.z; every block sums the partials itself
// (same order in every block), so no separate scalar kernels are needed.  Once
// converged (|r|^2 <= thr) every kernel returns early.
enum { CG_RZ = 0, CG_RR, CG_THR, CG_DONE, CG_IT, CG_ALPHA, CG_BETA, CG_NS };

__device__ __forceinline__ double block_sum(const double* part, int np, double* red) {
  double s = 0;
  for (int i = threadIdx.x; i < np; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double v = red[0];
  __syncthreads();
  return v;
}
// ---- rigid rotations (free slip on both spheres) -------------------------------
// Moments sum_i X_i x v_i of a velocity over the P2 nodes: FP64 partial sums
// per block, component k at partial[k * DOT_BLOCKS + block].
template <typename R>
__global__ __launch_bounds__(256) void k_rot_moment(const double* __restrict__ X, const R* __restrict__ v, long long n2,
                                                    double* __restrict__ partial) {
  __shared__ double red[3][256];
  double a = 0, b = 0, c = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n2; i += (long long)gridDim.x * blockDim.x) {
    const double x = X[3 * i], y = X[3 * i + 1], z = X[3 * i + 2];
    const double u = (double)v[i], w = (double)v[i + n2], q = (double)v[i + 2 * n2];
    a += y * q - z * w;
    b += z * u - x * q;
    c += x * w - y * u;
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  red[2][threadIdx.x] = c;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
#pragma unroll
      for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 3; ++k) partial[k * DOT_BLOCKS + blockIdx.x] = red[k][0];
  }
}
// v_i -= w x X_i, w = G^-1 m: every block sums the moment partials itself, in
// the same order, so no separate scalar kernel is needed.
template <typename R>
__global__ __launch_bounds__(256) void k_rot_remove(RotDev rd, long long n2, R* __restrict__ v,
                                                    const double* __restrict__ partial, int np);

__device__ __forceinline__ void block_partials(double a, double b, double* pa, double* pb, double (*red)[256]) {
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      red[0][threadIdx.x] += red[0][threadIdx.x + o];
      red[1][threadIdx.x] += red[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pa[blockIdx.x] = red[0][0];
    pb[blockIdx.x] = red[1][0];
  }
}
// v -= mean(v) on the device: per-block partial sums of v, then every block of
// the second kernel sums them itself (same order) and subtracts the mean
template <typename R>
__global__ __launch_bounds__(256) void k_sum_partials(const R* __restrict__ v, long long n, double* __restrict__ partial) {
  __shared__ double red[256];
  double a = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    a += (double)v[i];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}
template <typename R>
__global__ __launch_bounds__(256) void k_sub_mean(R* __restrict__ v, long long n, const double* __restrict__ partial,
                                                  int np) {
  __shared__ double red[256];
  const double mean = block_sum(partial, np, red) / (double)n;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    v[i] = R((double)v[i] - mean);
}

template <typename R>
__global__ __launch_bounds__(256) void k_rot_remove(RotDev rd, long long n2, R* __restrict__ v,
                                                    const double* __restrict__ partial, int np) {
  __shared__ double red[256];
  double m[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) m[k] = block_sum(partial + k * DOT_BLOCKS, np, red);
  double w[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) w[k] = rd.gi[3 * k] * m[0] + rd.gi[3 * k + 1] * m[1] + rd.gi[3 * k + 2] * m[2];
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n2; i += (long long)gridDim.x * blockDim.x) {
    const double x = rd.X[3 * i], y = rd.X[3 * i + 1], z = rd.X[3 * i + 2];
    v[i] = R((double)v[i] - (w[1] * z - w[2] * y));
    v[i + n2] = R((double)v[i + n2] - (w[2] * x - w[0] * z));
    v[i + 2 * n2] = R((double)v[i + 2 * n2] - (w[0] * y - w[1] * x));
  }
}

__device__ __forceinline__ double* cg_rr(double* part, int parity) { return part + DOT_BLOCKS + 2 * DOT_BLOCKS * parity; }
__device__ __forceinline__ double* cg_rz(double* part, int parity) { return cg_rr(part, parity) + DOT_BLOCKS; }
__device__ __forceinline__ const double* cg_rr(const double* part, int parity) {
  return part + DOT_BLOCKS + 2 * DOT_BLOCKS * parity;
}
__device__ __forceinline__ const double* cg_rz(const double* part, int parity) { return cg_rr(part, parity) + DOT_BLOCKS; }

template <typename R>
__global__ __launch_bounds__(256) void k_cg_init(const R* __restrict__ r, const R* __restrict__ dinv,
                                                 R* __restrict__ z, long long n, double* part) {
  __shared__ double red[2][256];
  double a = 0, b = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const R zi = dinv[i] * r[i];
    z[i] = zi;
    a += (double)r[i] * (double)r[i];
    b += (double)r[i] * (double)zi;
  }
  block_partials(a, b, cg_rr(part, 1), cg_rz(part, 1), red);   // "previous" parity of iteration 0
}

__global__ __launch_bounds__(256) void k_cg_init_fin(double* part, int np, double tol2, double* sc) {
  __shared__ double red[256];
  const double rr = block_sum(cg_rr(part, 1), np, red);
  const double rz = block_sum(cg_rz(part, 1), np, red);
  if (threadIdx.x == 0) {
    sc[CG_RR] = rr;
    sc[CG_RZ] = rz;
    sc[CG_THR] = tol2 * rr;
    sc[CG_DONE] = (rr == 0.0) ? 1.0 : 0.0;
    sc[CG_IT] = 0.0;
  }
}

// partials of p.q
template <typename R>
__global__ __launch_bounds__(256) void k_cg_dot(const double* sc, const R* __restrict__ x, const R* __restrict__ y,
                                                long long n, double* part) {
  if (sc[CG_DONE] != 0.0) return;
  __shared__ double red[256];
  double s = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    s += (double)x[i] * (double)y[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// alpha = r.z / p.q;  x += alpha p;  r -= alpha q;  z = D^-1 r;  partials of r.r, r.z
template <typename R>
__global__ __launch_bounds__(256) void k_cg_update(const double* sc, const R* __restrict__ p, const R* __restrict__ q,
                                                   const R* __restrict__ dinv, R* __restrict__ x, R* __restrict__ r,
                                                   R* __restrict__ z, long long n, double* part, int np, int parity) {
  if (sc[CG_DONE] != 0.0) return;
  __shared__ double red[2][256];
  const double pq = block_sum(part, np, red[0]);
  const double rz = block_sum(cg_rz(part, parity ^ 1), np, red[0]);
  const R alpha = R(rz / pq);
  double a = 0, b = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    x[i] += alpha * p[i];
    const R ri = r[i] - alpha * q[i];
    r[i] = ri;
    const R zi = dinv[i] * ri;
    z[i] = zi;
    a += (double)ri * (double)ri;
    b += (double)ri * (double)zi;
  }
  block_partials(a, b, cg_rr(part, parity), cg_rz(part, parity), red);
}

// convergence test; beta = r.z / previous r.z;  p = z + beta p
template <typename R>
__global__ __launch_bounds__(256) void k_cg_p(double* sc, const R* __restrict__ z, R* __restrict__ p, long long n,
                                              double* part, int np, int parity) {
  if (sc[CG_DONE] != 0.0) return;
  __shared__ double red[256];
  const double rr = block_sum(cg_rr(part, parity), np, red);
  const double rz = block_sum(cg_rz(part, parity), np, red);
  const double rzo = block_sum(cg_rz(part, parity ^ 1), np, red);
  const bool done = rr <= sc[CG_THR];
  __syncthreads();   // every block has read the scalars before block 0 updates them
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc[CG_IT] += 1.0;
    sc[CG_RR] = rr;
    sc[CG_RZ] = rz;
  }
  if (done) {
    if (blockIdx.x == 0 && threadIdx.x == 0) sc[CG_DONE] = 1.0;
    return;
  }
  const R beta = R(rz / rzo);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = z[i] + beta * p[i];
}

// ---- coarsest level: CG on stored element matrices -----------------------------
// The coarse solve (Sec. 5.2.2) runs many short iterations on a small level,
// where the element kernel is one long FP64 latency chain per thread.  The
// level's element matrices are therefore formed once per viscosity field, and
// an iteration is three kernels: element products A_e z_e, a node pass that
// sums them over the incident elements, projects, and forms p = z + beta p and
// q = A p = A z + beta q, and a node pass for the x, r, z updates.  Node
// passes hold the three components of a node, so the projections need no
// kernel of their own.

// column j of A_e of every micro-tet e (one thread per (e, j)): the element
// operator applied to the j-th unit vector, no boundary projection.  DIAG:
// only the diagonal entry, summed into d at its global DoF.
template <bool BLEND, bool DIAG>
__global__ __launch_bounds__(256) void k_elem_cols(LevelDev L, const double* __restrict__ eta,
                                                   double* __restrict__ emat, float* __restrict__ ematf,
                                                   double* __restrict__ d) {
  using E = StokesElem<double, BLEND, F_A>;
  const long long gid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int n = L.n, m2 = 2 * n;
  const int ne = n * n * n;
  if (gid >= (long long)ne * L.nmacro * 30) return;
  const long long e = gid / 30;
  const int j = (int)(gid - e * 30);
  const int mac = (int)(e / ne);
  const int pk = L.eall[e - (long long)mac * ne];
  const int type = pk & 7, px = (pk >> 3) & 1023, py = (pk >> 13) & 1023, pz = pk >> 23;
  const uint32_t* l1 = L.l2g1 + (size_t)mac * L.nloc1;
  const uint32_t* l2 = L.l2g2 + (size_t)mac * L.nloc2;
  const double* G = L.geo + (size_t)mac * 16;
  size_t g1[4], g2[10];
  int I2[10], J2[10], K2[10];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int I = px + c_toff[type][v][0], J = py + c_toff[type][v][1], K = pz + c_toff[type][v][2];
    g1[v] = l1[lloc(I, J, K, n)];
    I2[v] = 2 * I;
    J2[v] = 2 * J;
    K2[v] = 2 * K;
  }
#pragma unroll
  for (int ed = 0; ed < 6; ++ed) {
    I2[4 + ed] = (I2[EV0(ed)] + I2[EV1(ed)]) >> 1;
    J2[4 + ed] = (J2[EV0(ed)] + J2[EV1(ed)]) >> 1;
    K2[4 + ed] = (K2[EV0(ed)] + K2[EV1(ed)]) >> 1;
  }
  const bool qpv = BLEND && L.qpv;
  if (DIAG || qpv) {
#pragma unroll
    for (int a = 0; a < 10; ++a) g2[a] = l2[lloc(I2[a], J2[a], K2[a], m2)];
  }
  double xv[4][3];
  if (BLEND) elem_vertices<double>(G, type, px, py, pz, n, xv);
  double etq[4] = {0, 0, 0, 0};
  if (qpv) {
    double T10[10];
#pragma unroll
    for (int a = 0; a < 10; ++a) T10[a] = L.T2[g2[a]];
    qp_viscosity<double>(L.vm, G, xv, T10, etq);
  }
  E el;
  el.load(
      L.tinv + ((size_t)mac * 6 + type) * 10, [&](int v, int k) { return xv[v][k]; },
      [&](int c, int a) { return c * 10 + a == j ? 1.0 : 0.0; },
      [&](int v, double& ev, double&, double&) { ev = qpv ? etq[v] : eta[g1[v]]; });
  el.template qp<0>(G);
  el.template qp<1>(G);
  el.template qp<2>(G);
  el.template qp<3>(G);
  if (DIAG) {
    el.store(
        [&](int c, int a, double v) {
          if (c * 10 + a == j) gadd(d + g2[a] + (size_t)c * L.n2, v);
        },
        [](int, double) {});
  } else {
    double* col = emat + (size_t)e * 900 + (size_t)j * 30;
    float* colf = ematf + (size_t)e * 900 + (size_t)j * 30;
    el.store(
        [&](int c, int a, double v) {
          col[c * 10 + a] = v;
          colf[c * 10 + a] = (float)v;
        },
        [](int, double) {});
  }
}

// P2 nodal values of the next coarser level: coarse lattice point (I,J,K) is
// fine point (2I,2J,2K) of the same macro
template <typename R>
__global__ void k_inject_p2(LevelDev Lc, LevelDev Lf, const R* __restrict__ vf, R* __restrict__ vc) {
  const int mac = blockIdx.y;
  const int m = 2 * Lc.n;
  for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < Lc.nloc2; l += gridDim.x * blockDim.x) {
    int K = 0;
    while (tetc(m) - tetc(m - K - 1) <= l) ++K;
    int r = l - (int)(tetc(m) - tetc(m - K));
    const int s = m - K;
    int J = 0;
    while (r >= s - J + 1) { r -= s - J + 1; ++J; }
    const int I = r;
    const size_t gc = Lc.l2g2[(size_t)mac * Lc.nloc2 + l];
    const size_t gf = Lf.l2g2[(size_t)mac * Lf.nloc2 + lloc(2 * I, 2 * J, 2 * K, 2 * m)];
    vc[gc] = vf[gf];   // shared nodes get the same value from every macro
  }
}

// eta(x_V, T(x_V)) at the P1 vertices of a blended level (vertex (I,J,K) is
// P2 point (2I,2J,2K); its radius is s at the reference point)
__global__ void k_eta_vertices(LevelDev L, double* __restrict__ eta1) {
  const int mac = blockIdx.y;
  const int n = L.n;
  const double* G = L.geo + (size_t)mac * 16;
  for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < L.nloc1; l += gridDim.x * blockDim.x) {
    int K = 0;
    while (tetc(n) - tetc(n - K - 1) <= l) ++K;
    int r = l - (int)(tetc(n) - tetc(n - K));
    const int s = n - K;
    int J = 0;
    while (r >= s - J + 1) { r -= s - J + 1; ++J; }
    const int I = r;
    double x[3];
    lattice_x<double>(G, I, J, K, n, x);
    const double rad = G[12] * x[0] + G[13] * x[1] + G[14] * x[2] + G[15];
    const double T = L.T2[L.l2g2[(size_t)mac * L.nloc2 + lloc(2 * I, 2 * J, 2 * K, 2 * n)]];
    eta1[L.l2g1[(size_t)mac * L.nloc1 + l]] = visc_model<double>(L.vm, rad, T);
  }
}

__device__ __forceinline__ void node_project(int act, const double* __restrict__ nrm, double v[3]) {
  if (act == ACT_DIR) {
    v[0] = v[1] = v[2] = 0.0;
  } else if (act == ACT_FS) {
    const double dn = v[0] * nrm[0] + v[1] * nrm[1] + v[2] * nrm[2];
    v[0] -= dn * nrm[0];
    v[1] -= dn * nrm[1];
    v[2] -= dn * nrm[2];
  }
}

// Sums of up to three partial arrays in one pass (same order in every block).
__device__ __forceinline__ void block_sum3(const double* a, const double* b, const double* c, int np,
                                           double (*red)[256], double out[3]) {
  double s0 = 0, s1 = 0, s2 = 0;
  for (int i = threadIdx.x; i < np; i += 256) {
    s0 += a[i];
    if (b) s1 += b[i];
    if (c) s2 += c[i];
  }
  red[0][threadIdx.x] = s0;
  red[1][threadIdx.x] = s1;
  red[2][threadIdx.x] = s2;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      red[0][threadIdx.x] += red[0][threadIdx.x + o];
      red[1][threadIdx.x] += red[1][threadIdx.x + o];
      red[2][threadIdx.x] += red[2][threadIdx.x + o];
    }
    __syncthreads();
  }
  out[0] = red[0][0];
  out[1] = red[1][0];
  out[2] = red[2][0];
  __syncthreads();
}

// x = 0; r = P b; z = P D^-1 r; partials of r.r and r.z as the "previous" parity
__global__ __launch_bounds__(256) void k_ccg_init(CoarseDev cd, const double* __restrict__ b, double* __restrict__ x,
                                                  double* __restrict__ r, double* __restrict__ z, double* part) {
  __shared__ double red[2][256];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nn = (size_t)cd.nn;
  double a = 0, bb = 0;
  if (i < cd.nn) {
    double rv[3], zv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) rv[c] = b[i + c * nn];
    node_project(cd.act[i], cd.nrm + 3 * (size_t)i, rv);
#pragma unroll
    for (int c = 0; c < 3; ++c) zv[c] = cd.dinv[i + c * nn] * rv[c];
    node_project(cd.act[i], cd.nrm + 3 * (size_t)i, zv);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      x[i + c * nn] = 0.0;
      r[i + c * nn] = rv[c];
      z[i + c * nn] = zv[c];
      a += rv[c] * rv[c];
      bb += rv[c] * zv[c];
    }
  }
  block_partials(a, bb, cg_rr(part, 1), cg_rz(part, 1), red);
}

// The iteration kernels are short dependent chains of memory accesses, so
// each issues every load that does not depend on the iteration's scalars
// before it waits for any, and only then tests the convergence flag (a
// finished solve stores nothing).

// (A_e z_e)_j: the search direction's product follows by linearity,
// A p = A z + beta A p_prev, so this kernel needs no scalar of the iteration.
// Results go to the incidence slot of (e, local node) in node order, so that
// the node pass reads each node's contributions contiguously.  CCG_ELEMS
// elements of 30 threads per 256-thread workgroup.
template <typename M>
__global__ __launch_bounds__(256) void k_ccg_elem(CoarseDev cd, const M* __restrict__ emat, const double* sc,
                                                  const double* __restrict__ z, double* __restrict__ Y) {
  __shared__ double ze[CCG_ELEMS][30];
  const int le = threadIdx.x / 30, j = threadIdx.x - 30 * le;
  const long long e = (long long)blockIdx.x * CCG_ELEMS + le;
  const bool on = le < CCG_ELEMS && e < cd.ne;
  const double done = sc[CG_DONE];
  double a[30];
  double zv = 0.0;
  size_t slot = 0;
  if (on) {
    const M* A = emat + (size_t)e * 900 + j;
#pragma unroll
    for (int k = 0; k < 30; ++k) a[k] = A[30 * k];
    zv = z[(size_t)cd.enode[e * 10 + j % 10] + (size_t)(j / 10) * cd.nn];
    slot = (size_t)cd.epos[e * 10 + j % 10] + (size_t)(j / 10) * ((size_t)cd.ne * 10);
  }
  if (done != 0.0) return;
  if (on) ze[le][j] = zv;
  __syncthreads();
  if (on) {
    double y = 0.0;
#pragma unroll
    for (int k = 0; k < 30; ++k) y = fma(a[k], ze[le][k], y);
    Y[slot] = y;
  }
}

// convergence test on |r|^2 of the previous iteration; beta = r.z / previous
// r.z; p = z + beta p; q = P A p = P (sum of the incident element rows of A z)
// + beta q; partials of p.q
__global__ __launch_bounds__(256) void k_ccg_node1(CoarseDev cd, double* sc, double* part, int np,
                                                   const double* __restrict__ z, double* __restrict__ p,
                                                   double* __restrict__ q, const double* __restrict__ Y, int parity,
                                                   int first) {
  __shared__ double red[3][256];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nn = (size_t)cd.nn;
  const bool on = i < cd.nn;
  const double done = sc[CG_DONE], thr = sc[CG_THR];
  double zv[3] = {0, 0, 0}, po[3] = {0, 0, 0}, qo[3] = {0, 0, 0}, qv[3] = {0, 0, 0}, nr[3] = {0, 0, 0};
  int act = ACT_NONE;
  if (on) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const size_t g = i + c * nn;
      zv[c] = z[g];
      po[c] = p[g];
      qo[c] = q[g];
      nr[c] = cd.nrm[3 * (size_t)i + c];
    }
    act = cd.act[i];
    const int k0 = cd.iptr[i], k1 = cd.iptr[i + 1];
    const size_t ninc = (size_t)cd.ne * 10;
    for (int kb = k0; kb < k1; kb += 8) {
      // branch-free batch: every load of the batch is in flight at once
      // (slots past the node's list read slot k0 and are weighted 0)
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int k = kb + u < k1 ? kb + u : k0;
        const double w = kb + u < k1 ? 1.0 : 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) qv[c] = fma(w, Y[k + c * ninc], qv[c]);
      }
    }
  }
  double sums[3] = {0, 0, 0};   // |r|^2, r.z, previous r.z
  if (!first) block_sum3(cg_rr(part, parity ^ 1), cg_rz(part, parity ^ 1), cg_rz(part, parity), np, red, sums);
  if (done != 0.0) return;
  if (!first && sums[0] <= thr) {
    if (blockIdx.x == 0 && threadIdx.x == 0) sc[CG_DONE] = 1.0;
    return;
  }
  const double beta = first ? 0.0 : sums[1] / sums[2];
  double s = 0;
  if (on) {
    node_project(act, nr, qv);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const size_t g = i + c * nn;
      const double pv = first ? zv[c] : fma(beta, po[c], zv[c]);
      const double qc = first ? qv[c] : fma(beta, qo[c], qv[c]);
      p[g] = pv;
      q[g] = qc;
      s += pv * qc;
    }
  }
  red[0][threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[0][threadIdx.x] += red[0][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0][0];
}

// alpha = r.z / p.q; x += alpha p; r -= alpha q; z = P D^-1 r; partials of
// r.r and r.z of this parity; iteration count
__global__ __launch_bounds__(256) void k_ccg_node2(CoarseDev cd, double* sc, double* part, int np,
                                                   const double* __restrict__ p, const double* __restrict__ q,
                                                   double* __restrict__ x, double* __restrict__ r,
                                                   double* __restrict__ z, int parity) {
  __shared__ double red[3][256];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nn = (size_t)cd.nn;
  const bool on = i < cd.nn;
  const double done = sc[CG_DONE];
  double pv[3] = {0, 0, 0}, qv[3] = {0, 0, 0}, xv[3] = {0, 0, 0}, rv[3] = {0, 0, 0}, dv[3] = {0, 0, 0},
         nr[3] = {0, 0, 0};
  int act = ACT_NONE;
  if (on) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const size_t g = i + c * nn;
      pv[c] = p[g];
      qv[c] = q[g];
      xv[c] = x[g];
      rv[c] = r[g];
      dv[c] = cd.dinv[g];
      nr[c] = cd.nrm[3 * (size_t)i + c];
    }
    act = cd.act[i];
  }
  double sums[3];   // p.q, previous r.z
  block_sum3(part, cg_rz(part, parity ^ 1), nullptr, np, red, sums);
  if (done != 0.0) return;
  const double alpha = sums[1] / sums[0];
  double a = 0, b = 0;
  if (on) {
    double zv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      xv[c] += alpha * pv[c];
      rv[c] -= alpha * qv[c];
      zv[c] = dv[c] * rv[c];
    }
    node_project(act, nr, zv);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const size_t g = i + c * nn;
      x[g] = xv[c];
      r[g] = rv[c];
      z[g] = zv[c];
      a += rv[c] * rv[c];
      b += rv[c] * zv[c];
    }
  }
  block_partials(a, b, cg_rr(part, parity), cg_rz(part, parity), reinterpret_cast<double (*)[256]>(red));
  if (blockIdx.x == 0 && threadIdx.x == 0) sc[CG_IT] += 1.0;
}

void launch_elem_matrix(const LevelDev& L, const double* eta, double* emat, float* ematf, hipStream_t s) {
  const long long tot = (long long)L.n * L.n * L.n * L.nmacro * 30;
  dim3 grid((unsigned)((tot + 255) / 256));
  if (L.blend) hipLaunchKernelGGL((k_elem_cols<true, false>), grid, dim3(256), 0, s, L, eta, emat, ematf, nullptr);
  else hipLaunchKernelGGL((k_elem_cols<false, false>), grid, dim3(256), 0, s, L, eta, emat, ematf, nullptr);
}
void launch_elem_diag(const LevelDev& L, const double* eta, double* d, hipStream_t s) {
  const long long tot = (long long)L.n * L.n * L.n * L.nmacro * 30;
  dim3 grid((unsigned)((tot + 255) / 256));
  if (L.blend) hipLaunchKernelGGL((k_elem_cols<true, true>), grid, dim3(256), 0, s, L, eta, nullptr, nullptr, d);
  else hipLaunchKernelGGL((k_elem_cols<false, true>), grid, dim3(256), 0, s, L, eta, nullptr, nullptr, d);
}
void launch_eta_vertices(const LevelDev& L, double* eta1, hipStream_t s) {
  dim3 grid((unsigned)((L.nloc1 + 255) / 256), (unsigned)L.nmacro);
  hipLaunchKernelGGL(k_eta_vertices, grid, dim3(256), 0, s, L, eta1);
}
template <typename R>
void launch_inject_p2(const LevelDev& Lc, const LevelDev& Lf, const R* vf, R* vc, hipStream_t s) {
  dim3 grid((unsigned)((Lc.nloc2 + 255) / 256), (unsigned)Lc.nmacro);
  hipLaunchKernelGGL((k_inject_p2<R>), grid, dim3(256), 0, s, Lc, Lf, vf, vc);
}
template void launch_inject_p2<double>(const LevelDev&, const LevelDev&, const double*, double*, hipStream_t);
void ccg_init(const CoarseDev& cd, const double* b, double* x, double* r, double* z, double tol, double* part,
              double* sc, hipStream_t s) {
  const int nb = (cd.nn + 255) / 256;
  hipLaunchKernelGGL(k_ccg_init, dim3(nb), dim3(256), 0, s, cd, b, x, r, z, part);
  hipLaunchKernelGGL(k_cg_init_fin, dim3(1), dim3(256), 0, s, part, nb, tol * tol, sc);
}
void ccg_iter(const CoarseDev& cd, bool fp32, double* x, double* r, double* z, double* p, double* q, double* Y,
              double* part, double* sc, int it, hipStream_t s) {
  const int nb = (cd.nn + 255) / 256, parity = it & 1, first = it == 0;
  const dim3 ge((cd.ne + CCG_ELEMS - 1) / CCG_ELEMS);
  if (fp32) hipLaunchKernelGGL(k_ccg_elem<float>, ge, dim3(256), 0, s, cd, cd.ematf, sc, z, Y);
  else hipLaunchKernelGGL(k_ccg_elem<double>, ge, dim3(256), 0, s, cd, cd.emat, sc, z, Y);
  hipLaunchKernelGGL(k_ccg_node1, dim3(nb), dim3(256), 0, s, cd, sc, part, nb, z, p, q, Y, parity, first);
  hipLaunchKernelGGL(k_ccg_node2, dim3(nb), dim3(256), 0, s, cd, sc, part, nb, p, q, x, r, z, parity);
}

static inline int redgrid(long long n) {
  long long g = (n + 255) / 256;
  return (int)(g < DOT_BLOCKS ? (g < 1 ? 1 : g) : DOT_BLOCKS);
}

template <typename R>
void cg_init(const R* r, const R* dinv, R* z, long long n, double tol, double* part, double* sc, hipStream_t s) {
  const int nb = redgrid(n);
  hipLaunchKernelGGL((k_cg_init<R>), dim3(nb), dim3(256), 0, s, r, dinv, z, n, part);
  hipLaunchKernelGGL(k_cg_init_fin, dim3(1), dim3(256), 0, s, part, nb, tol * tol, sc);
}
template <typename R>
void cg_dot(const R* p, const R* q, long long n, double* part, const double* sc, hipStream_t s) {
  hipLaunchKernelGGL((k_cg_dot<R>), dim3(redgrid(n)), dim3(256), 0, s, sc, p, q, n, part);
}
template <typename R>
void cg_update(const R* p, const R* q, const R* dinv, R* x, R* r, R* z, long long n, double* part, const double* sc,
               int parity, hipStream_t s) {
  const int nb = redgrid(n);
  hipLaunchKernelGGL((k_cg_update<R>), dim3(nb), dim3(256), 0, s, sc, p, q, dinv, x, r, z, n, part, nb, parity);
}
template <typename R>
void cg_pupdate(const R* z, R* p, long long n, double* part, double* sc, int parity, hipStream_t s) {
  const int nb = redgrid(n);
  hipLaunchKernelGGL((k_cg_p<R>), dim3(nb), dim3(256), 0, s, sc, z, p, n, part, nb, parity);
}
#define INST_CG(R)                                                                                                \
  template void cg_init<R>(const R*, const R*, R*, long long, double, double*, double*, hipStream_t);           \
  template void cg_dot<R>(const R*, const R*, long long, double*, const double*, hipStream_t);                 \
  template void cg_update<R>(const R*, const R*, const R*, R*, R*, R*, long long, double*, const double*, int,  \
                             hipStream_t);                                                                      \
  template void cg_pupdate<R>(const R*, R*, long long, double*, double*, int, hipStream_t);

// ---- launch wrappers ----------------------------------------------------------------
static inline int vgrid(long long n) {
  long long g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}

size_t sweep_lds_bytes(int FL, int cap2, int cap1, int rb) { return sweep_lds(FL, cap2, cap1, rb).total; }

template <typename R, int FL>
static void stokes_dispatch(const LevelDev& L, const R* u, const R* p, const R* eta, const R* lnrho, R* yu, R* yp,
                            R* sl2, R* sl1, int bcmode, hipStream_t s) {
  if (L.elemwise) {
    constexpr bool OU = FL & (F_A | F_BT | F_CT), OP = FL & (F_B | F_C | F_M);
    if (OU) vfill<R>(yu, R(0), 3 * L.n2, s);
    if (OP) vfill<R>(yp, R(0), L.n1, s);
    const long long tot = (long long)L.n * L.n * L.n * L.nmacro;
    dim3 grid((unsigned)((tot + 255) / 256));
    if (L.blend)
      hipLaunchKernelGGL((k_elemwise<R, true, FL>), grid, dim3(256), 0, s, L, u, p, eta, lnrho, yu, yp, bcmode);
    else
      hipLaunchKernelGGL((k_elemwise<R, false, FL>), grid, dim3(256), 0, s, L, u, p, eta, lnrho, yu, yp, bcmode);
    return;
  }
  dim3 grid((unsigned)(L.sw.nstrips * L.nmacro));
  const size_t lds = sweep_lds_bytes(FL, L.sw.cap2, L.sw.cap1, sizeof(R));
  // a layer of a macro holds about n^2 micro-tets: smaller workgroups on the
  // coarser levels keep the threads busy and let more macros run per CU
  const unsigned bsz = L.n <= 4 ? 64 : (L.n <= 8 ? 128 : 256);
  if (L.blend)
    hipLaunchKernelGGL((k_sweep<R, true, FL>), grid, dim3(bsz), lds, s, L, u, p, eta, lnrho, yu, yp, sl2, sl1, bcmode);
  else
    hipLaunchKernelGGL((k_sweep<R, false, FL>), grid, dim3(bsz), lds, s, L, u, p, eta, lnrho, yu, yp, sl2, sl1, bcmode);
}

template <typename R>
void launch_stokes(int flags, const LevelDev& L, const BcDev& bc, const R* u, const R* p, const R* eta,
                   const R* lnrho, R* yu, R* yp, R* sl2, R* sl1, int bcmode, hipStream_t s, hipEvent_t ev0,
                   hipEvent_t ev1) {
  if (ev0) (void)hipEventRecord(ev0, s);
  switch (flags) {
#define CASE(F) case F: stokes_dispatch<R, F>(L, u, p, eta, lnrho, yu, yp, sl2, sl1, bcmode, s); break;
    CASE(F_A)
    CASE(F_BT)
    CASE(F_BT | F_CT)
    CASE(F_B)
    CASE(F_B | F_C)
    CASE(F_M)
    CASE(F_A | F_BT)
    CASE(F_A | F_BT | F_B)
    CASE(F_A | F_BT | F_B | F_C)
    CASE(F_A | F_BT | F_CT | F_B)
#undef CASE
    default: return;
  }
  if (ev1) (void)hipEventRecord(ev1, s);
  const bool OU = flags & (F_A | F_BT | F_CT), OP = flags & (F_B | F_C | F_M);
  if (OU && L.g2.nnodes > 0 && !L.elemwise)
    hipLaunchKernelGGL((k_gather<R, 3>), dim3((L.g2.nnodes + 255) / 256), dim3(256), 0, s, L.g2, sl2,
                       (size_t)L.nmacro * L.sw.nsh2, yu, (size_t)L.n2);
  if (OP && L.g1.nnodes > 0 && !L.elemwise)
    hipLaunchKernelGGL((k_gather<R, 1>), dim3((L.g1.nnodes + 255) / 256), dim3(256), 0, s, L.g1, sl1,
                       (size_t)L.nmacro * L.sw.nsh1, yp, (size_t)L.n1);
  if (OU && (bcmode & BCM_OUT)) launch_project<R>(bc, L.n2, yu, s);
}
template void launch_stokes<double>(int, const LevelDev&, const BcDev&, const double*, const double*, const double*,
                                    const double*, double*, double*, double*, double*, int, hipStream_t, hipEvent_t,
                                    hipEvent_t);
template void launch_stokes<float>(int, const LevelDev&, const BcDev&, const float*, const float*, const float*,
                                   const float*, float*, float*, float*, float*, int, hipStream_t, hipEvent_t,
                                   hipEvent_t);

template <typename R>
void launch_diag(const LevelDev& L, const R* eta, R* d, hipStream_t s) {
  dim3 grid((unsigned)(L.ntiles * L.nmacro));
  if (L.blend) hipLaunchKernelGGL((k_diag<R, true>), grid, dim3(384), 0, s, L, eta, d);
  else hipLaunchKernelGGL((k_diag<R, false>), grid, dim3(384), 0, s, L, eta, d);
}
template void launch_diag<double>(const LevelDev&, const double*, double*, hipStream_t);
template void launch_diag<float>(const LevelDev&, const float*, float*, hipStream_t);

template <typename R>
void launch_mass_bricks(const LevelDev& L, const R* eta, const R* p, R* y, hipStream_t s) {
  dim3 grid((unsigned)(L.ntiles * L.nmacro));
  if (L.blend) hipLaunchKernelGGL((k_mass<R, true, false>), grid, dim3(384), 0, s, L, eta, p, y);
  else hipLaunchKernelGGL((k_mass<R, false, false>), grid, dim3(384), 0, s, L, eta, p, y);
}
template void launch_mass_bricks<double>(const LevelDev&, const double*, const double*, double*, hipStream_t);
template void launch_mass_bricks<float>(const LevelDev&, const float*, const float*, float*, hipStream_t);
void launch_mass_diag(const LevelDev& L, const double* eta, double* y, hipStream_t s) {
  dim3 grid((unsigned)(L.ntiles * L.nmacro));
  if (L.blend) hipLaunchKernelGGL((k_mass<double, true, true>), grid, dim3(384), 0, s, L, eta, nullptr, y);
  else hipLaunchKernelGGL((k_mass<double, false, true>), grid, dim3(384), 0, s, L, eta, nullptr, y);
}

void launch_mass_stencil_build(const LevelDev& L, const double* eta, double* c64, float* c32, hipStream_t s) {
  const long long nt = (long long)L.nloc1 * L.nmacro;
  dim3 grid((unsigned)((nt + 255) / 256));
  if (L.blend) hipLaunchKernelGGL((k_mass_stencil_build<true>), grid, dim3(256), 0, s, L, eta, c64, c32);
  else hipLaunchKernelGGL((k_mass_stencil_build<false>), grid, dim3(256), 0, s, L, eta, c64, c32);
}
size_t mass_stencil_lds_bytes(int nloc1, int real_bytes) { return ((size_t)nloc1 + 1) * real_bytes; }
template <typename R> static const R* mcoef_host(const LevelDev& L);
template <> const double* mcoef_host<double>(const LevelDev& L) { return L.ms.c64; }
template <> const float* mcoef_host<float>(const LevelDev& L) { return L.ms.c32; }
template <typename R>
void launch_mass_stencil(const LevelDev& L, const R* p, R* y, R* slots, hipStream_t s) {
  launch_stencil<R>(L, mcoef_host<R>(L), p, y, slots, s);
}
template <typename R>
void launch_stencil(const LevelDev& L, const R* coef, const R* p, R* y, R* slots, hipStream_t s) {
  hipLaunchKernelGGL((k_mass_stencil<R>), dim3((unsigned)L.nmacro), dim3(256),
                     mass_stencil_lds_bytes(L.nloc1, sizeof(R)), s, L, coef, p, y, slots);
  if (L.ms.g.nnodes > 0)
    hipLaunchKernelGGL((k_gather<R, 1>), dim3((L.ms.g.nnodes + 255) / 256), dim3(256), 0, s, L.ms.g, slots,
                       (size_t)0, y, (size_t)0);
}
template void launch_mass_stencil<double>(const LevelDev&, const double*, double*, double*, hipStream_t);
template void launch_mass_stencil<float>(const LevelDev&, const float*, float*, float*, hipStream_t);
template void launch_stencil<double>(const LevelDev&, const double*, const double*, double*, double*, hipStream_t);
template void launch_stencil<float>(const LevelDev&, const float*, const float*, float*, float*, hipStream_t);

void launch_rhs(const LevelDev& L, const double* T, double scale, double* f, hipStream_t s) {
  dim3 grid((unsigned)(L.ntiles * L.nmacro));
  if (L.blend)
    hipLaunchKernelGGL((k_rhs_grad<true, 0>), grid, dim3(384), 0, s, L, T, nullptr, nullptr, nullptr, f, nullptr, scale);
  else
    hipLaunchKernelGGL((k_rhs_grad<false, 0>), grid, dim3(384), 0, s, L, T, nullptr, nullptr, nullptr, f, nullptr, scale);
}
void launch_gradient(const LevelDev& L, const double* eta, const double* u, const double* lam, double* gm, double* gT,
                     double scale, hipStream_t s) {
  dim3 grid((unsigned)(L.ntiles * L.nmacro));
  if (L.blend)
    hipLaunchKernelGGL((k_rhs_grad<true, 1>), grid, dim3(384), 0, s, L, nullptr, u, lam, eta, gT, gm, scale);
  else
    hipLaunchKernelGGL((k_rhs_grad<false, 1>), grid, dim3(384), 0, s, L, nullptr, u, lam, eta, gT, gm, scale);
}

template <typename R>
void launch_prolong(const LevelDev& Lc, const LevelDev& Lf, const R* ec, R* ef, int bcmode, hipStream_t s) {
  dim3 grid((unsigned)(Lc.ntiles * Lc.nmacro));
  hipLaunchKernelGGL((k_transfer<R, 0>), grid, dim3(256), 0, s, Lc, Lf, ec, nullptr, ef, bcmode);
}
template <typename R>
void launch_restrict(const LevelDev& Lc, const LevelDev& Lf, const R* rf, R* rc, int bcmode, hipStream_t s) {
  dim3 grid((unsigned)(Lc.ntiles * Lc.nmacro));
  hipLaunchKernelGGL((k_transfer<R, 1>), grid, dim3(256), 0, s, Lc, Lf, rf, nullptr, rc, bcmode);
}
template <typename R>
void launch_prolong_add(const LevelDev& Lc, const LevelDev& Lf, const R* ec, R* ef, int bcmode, hipStream_t s) {
  dim3 grid((unsigned)(Lc.ntiles * Lc.nmacro));
  hipLaunchKernelGGL((k_transfer<R, 2>), grid, dim3(256), 0, s, Lc, Lf, ec, nullptr, ef, bcmode);
}
template <typename R>
void launch_restrict_diff(const LevelDev& Lc, const LevelDev& Lf, const R* bf, const R* tf, R* rc, int bcmode,
                          hipStream_t s) {
  dim3 grid((unsigned)(Lc.ntiles * Lc.nmacro));
  hipLaunchKernelGGL((k_transfer<R, 3>), grid, dim3(256), 0, s, Lc, Lf, bf, tf, rc, bcmode);
}
template void launch_prolong_add<double>(const LevelDev&, const LevelDev&, const double*, double*, int, hipStream_t);
template void launch_prolong_add<float>(const LevelDev&, const LevelDev&, const float*, float*, int, hipStream_t);
template void launch_restrict_diff<double>(const LevelDev&, const LevelDev&, const double*, const double*, double*,
                                           int, hipStream_t);
template void launch_restrict_diff<float>(const LevelDev&, const LevelDev&, const float*, const float*, float*, int,
                                          hipStream_t);
template void launch_prolong<double>(const LevelDev&, const LevelDev&, const double*, double*, int, hipStream_t);
template void launch_prolong<float>(const LevelDev&, const LevelDev&, const float*, float*, int, hipStream_t);
template void launch_restrict<double>(const LevelDev&, const LevelDev&, const double*, double*, int, hipStream_t);
template void launch_restrict<float>(const LevelDev&, const LevelDev&, const float*, float*, int, hipStream_t);

template <typename R>
void launch_inject(const LevelDev& Lc, const LevelDev& Lf, const R* vf, R* vc, hipStream_t s) {
  dim3 grid((unsigned)((Lc.nloc1 + 255) / 256), (unsigned)Lc.nmacro);
  hipLaunchKernelGGL((k_inject<R>), grid, dim3(256), 0, s, Lc, Lf, vf, vc);
}
template void launch_inject<double>(const LevelDev&, const LevelDev&, const double*, double*, hipStream_t);
template void launch_inject<float>(const LevelDev&, const LevelDev&, const float*, float*, hipStream_t);

template <typename R>
void launch_project(const BcDev& bc, long long n2, R* v, hipStream_t s) {
  const int n = bc.ndir + bc.nfs;
  if (n == 0) return;
  hipLaunchKernelGGL((k_project<R>), dim3((n + 255) / 256), dim3(256), 0, s, bc, n2, v);
}
template <typename R>
void launch_rot_remove(const RotDev& rd, long long n2, R* v, double* partial, hipStream_t s) {
  // at most DOT_BLOCKS blocks: the partial buffer holds DOT_BLOCKS per component,
  // and every block of the second kernel sums all of them
  const int nb = vgrid(n2) < DOT_BLOCKS ? vgrid(n2) : DOT_BLOCKS;
  hipLaunchKernelGGL((k_rot_moment<R>), dim3(nb), dim3(256), 0, s, rd.X, v, n2, partial);
  hipLaunchKernelGGL((k_rot_remove<R>), dim3(nb), dim3(256), 0, s, rd, n2, v, partial, nb);
}
template <typename R>
void launch_remove_mean(R* v, long long n, double* partial, hipStream_t s) {
  const int nb = vgrid(n) < DOT_BLOCKS ? vgrid(n) : DOT_BLOCKS;
  hipLaunchKernelGGL((k_sum_partials<R>), dim3(nb), dim3(256), 0, s, v, n, partial);
  hipLaunchKernelGGL((k_sub_mean<R>), dim3(nb), dim3(256), 0, s, v, n, partial, nb);
}
template void launch_remove_mean<double>(double*, long long, double*, hipStream_t);
template void launch_remove_mean<float>(float*, long long, double*, hipStream_t);
template void launch_rot_remove<double>(const RotDev&, long long, double*, double*, hipStream_t);
template void launch_rot_remove<float>(const RotDev&, long long, float*, double*, hipStream_t);
template void launch_project<double>(const BcDev&, long long, double*, hipStream_t);
template void launch_project<float>(const BcDev&, long long, float*, hipStream_t);

template <typename R> void vfill(R* x, R a, long long n, hipStream_t s) { hipLaunchKernelGGL((k_fill<R>), dim3(vgrid(n)), dim3(256), 0, s, x, a, n); }
template <typename R> void vcopy(const R* x, R* y, long long n, hipStream_t s) { hipLaunchKernelGGL((k_copy<R>), dim3(vgrid(n)), dim3(256), 0, s, x, y, n); }
template <typename R> void vaxpy(R a, const R* x, R* y, long long n, hipStream_t s) { hipLaunchKernelGGL((k_axpy<R>), dim3(vgrid(n)), dim3(256), 0, s, a, x, y, n); }
template <typename R> void vaxpby(R a, const R* x, R b, R* y, long long n, hipStream_t s) { hipLaunchKernelGGL((k_axpby<R>), dim3(vgrid(n)), dim3(256), 0, s, a, x, b, y, n); }
template <typename R> void vscale(R a, R* x, long long n, hipStream_t s) { hipLaunchKernelGGL((k_scale<R>), dim3(vgrid(n)), dim3(256), 0, s, a, x, n); }
template <typename R> void vmul(const R* a, const R* x, R* y, long long n, hipStream_t s) { hipLaunchKernelGGL((k_mul<R>), dim3(vgrid(n)), dim3(256), 0, s, a, x, y, n); }
template <typename A, typename B> void vconvert(const A* x, B* y, long long n, hipStream_t s) { hipLaunchKernelGGL((k_convert<A, B>), dim3(vgrid(n)), dim3(256), 0, s, x, y, n); }
template <typename R> void vinvert(const R* d, R* y, long long n, hipStream_t s) { hipLaunchKernelGGL((k_invert<R>), dim3(vgrid(n)), dim3(256), 0, s, d, y, n); }
void vexp(const double* x, double* y, long long n, hipStream_t s) { hipLaunchKernelGGL(k_exp, dim3(vgrid(n)), dim3(256), 0, s, x, y, n); }
template <typename R> void vcheb_start(const R* b, const R* t, const R* dinv, R c1, R* r, R* d, long long n, hipStream_t s) {
  hipLaunchKernelGGL((k_cheb_start<R>), dim3(vgrid(n)), dim3(256), 0, s, b, t, dinv, c1, r, d, n);
}
template <typename R> void vcheb_one(const R* b, const R* t, const R* dinv, R c1, R* x, bool xin, long long n, hipStream_t s) {
  hipLaunchKernelGGL((k_cheb_one<R>), dim3(vgrid(n)), dim3(256), 0, s, b, t, dinv, c1, x, (int)xin, n);
}
template <typename R> void vcheb_step(const R* t, const R* dinv, R c1, R c2, R* r, R* x, R* d, bool xin, long long n, hipStream_t s) {
  hipLaunchKernelGGL((k_cheb_step<R>), dim3(vgrid(n)), dim3(256), 0, s, t, dinv, c1, c2, r, x, d, (int)xin, n);
}
template <typename R> void vcheb_last(const R* t, const R* dinv, R c1, R c2, const R* r, const R* d, R* x, bool xin, long long n, hipStream_t s) {
  hipLaunchKernelGGL((k_cheb_last<R>), dim3(vgrid(n)), dim3(256), 0, s, t, dinv, c1, c2, r, d, x, (int)xin, n);
}
template <typename R> void vsub(const R* b, const R* t, R* r, long long n, hipStream_t s) {
  hipLaunchKernelGGL((k_sub<R>), dim3(vgrid(n)), dim3(256), 0, s, b, t, r, n);
}
template <typename R> void vdot(const R* x, const R* y, long long n, double* partial, double* out, hipStream_t s) {
  long long g = (n + 255) / 256;
  int nb = (int)(g < DOT_BLOCKS ? (g < 1 ? 1 : g) : DOT_BLOCKS);
  hipLaunchKernelGGL((k_dot<R>), dim3(nb), dim3(256), 0, s, x, y, n, partial);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, partial, nb, out);
}
template <typename R>
void vaxpy2_nrm(R a, const R* p, R* x, R b, const R* q, R* r, long long n, double* partial, double* out, hipStream_t s) {
  long long g = (n + 255) / 256;
  int nb = (int)(g < DOT_BLOCKS ? (g < 1 ? 1 : g) : DOT_BLOCKS);
  hipLaunchKernelGGL((k_axpy2_nrm<R>), dim3(nb), dim3(256), 0, s, a, p, x, b, q, r, n, partial);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, partial, nb, out);
}
void vsum_partials(double* partial, int np, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, partial, np, out);
}

void launch_poisson_stencil_build(const LevelDev& L, const double* eta, double a2, double* c64, float* c32,
                                  hipStream_t s) {
  const long long nt = (long long)L.nloc1 * L.nmacro;
  dim3 grid((unsigned)((nt + 255) / 256));
  if (L.blend) hipLaunchKernelGGL((k_poisson_stencil_build<true>), grid, dim3(256), 0, s, L, eta, a2, c64, c32);
  else hipLaunchKernelGGL((k_poisson_stencil_build<false>), grid, dim3(256), 0, s, L, eta, a2, c64, c32);
}
template <typename R>
void launch_stencil_diag(const LevelDev& L, const double* c64, R* d, hipStream_t s) {
  const long long nt = (long long)L.nloc1 * L.nmacro;
  vfill<R>(d, R(0), L.n1, s);
  hipLaunchKernelGGL((k_stencil_diag<R>), dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, L, c64, d);
}
template void launch_stencil_diag<double>(const LevelDev&, const double*, double*, hipStream_t);
template void launch_stencil_diag<float>(const LevelDev&, const double*, float*, hipStream_t);
template <typename R>
void launch_p1_prolong(const LevelDev& Lc, const LevelDev& Lf, const R* ec, R* ef, hipStream_t s) {
  const long long nt = (long long)Lf.nloc1 * Lf.nmacro;
  hipLaunchKernelGGL((k_p1_transfer<R, 0>), dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, Lc, Lf, ec, ef);
}
template <typename R>
void launch_p1_restrict(const LevelDev& Lc, const LevelDev& Lf, const R* rf, R* rc, hipStream_t s) {
  const long long nt = (long long)Lf.nloc1 * Lf.nmacro;
  vfill<R>(rc, R(0), Lc.n1, s);
  hipLaunchKernelGGL((k_p1_transfer<R, 1>), dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, Lc, Lf, rf, rc);
}
template void launch_p1_prolong<double>(const LevelDev&, const LevelDev&, const double*, double*, hipStream_t);
template void launch_p1_prolong<float>(const LevelDev&, const LevelDev&, const float*, float*, hipStream_t);
template void launch_p1_restrict<double>(const LevelDev&, const LevelDev&, const double*, double*, hipStream_t);
template void launch_p1_restrict<float>(const LevelDev&, const LevelDev&, const float*, float*, hipStream_t);
template <typename R>
void launch_vmass(const LevelDev& L, const VmassRule& qr, const R* eta, R a2, const R* u, R* y, bool diag, int bcmode,
                  hipStream_t s) {
  const long long tot = (long long)L.n * L.n * L.n * L.nmacro;
  dim3 grid((unsigned)((tot + 255) / 256));
  vfill<R>(y, R(0), 3 * L.n2, s);
  if (L.blend) {
    if (diag) hipLaunchKernelGGL((k_vmass<R, true, true>), grid, dim3(256), 0, s, L, qr, eta, a2, u, y, bcmode);
    else hipLaunchKernelGGL((k_vmass<R, true, false>), grid, dim3(256), 0, s, L, qr, eta, a2, u, y, bcmode);
  } else {
    if (diag) hipLaunchKernelGGL((k_vmass<R, false, true>), grid, dim3(256), 0, s, L, qr, eta, a2, u, y, bcmode);
    else hipLaunchKernelGGL((k_vmass<R, false, false>), grid, dim3(256), 0, s, L, qr, eta, a2, u, y, bcmode);
  }
}
template void launch_vmass<double>(const LevelDev&, const VmassRule&, const double*, double, const double*, double*,
                                   bool, int, hipStream_t);

void launch_temp(const LevelDev& L, const VmassRule& qr, const TempCoef& tc, int mode, const double* x,
                 const double* u, const double* lnrho, const double* eta, const double* Tn, const double* Tm, double* y,
                 hipStream_t s) {
  const long long tot = (long long)L.n * L.n * L.n * L.nmacro;
  dim3 grid((unsigned)((tot + 255) / 256));
  vfill<double>(y, 0.0, L.n2, s);
#define TEMP_LAUNCH(M)                                                                                         \
  do {                                                                                                         \
    if (L.blend) hipLaunchKernelGGL((k_temp<M, true>), grid, dim3(256), 0, s, L, qr, tc, x, u, lnrho, eta, Tn, Tm, y); \
    else hipLaunchKernelGGL((k_temp<M, false>), grid, dim3(256), 0, s, L, qr, tc, x, u, lnrho, eta, Tn, Tm, y);        \
  } while (0)
  switch (mode) {
    case TM_APPLY: TEMP_LAUNCH(TM_APPLY); break;
    case TM_SYM: TEMP_LAUNCH(TM_SYM); break;
    case TM_DIAG: TEMP_LAUNCH(TM_DIAG); break;
    default: TEMP_LAUNCH(TM_RHS); break;
  }
#undef TEMP_LAUNCH
}

size_t temp_smat_slots(const LevelDev& L) { return (size_t)L.nmacro * L.ntiles * 384; }

void launch_temp_smat(const LevelDev& L, const VmassRule& qr, double s1, double tk, const double* lnrho, double* S,
                      hipStream_t s) {
  dim3 grid((unsigned)(L.nmacro * L.ntiles));
  if (L.blend) hipLaunchKernelGGL((k_temp_smat<true>), grid, dim3(384), 0, s, L, qr, s1, tk, lnrho, S);
  else hipLaunchKernelGGL((k_temp_smat<false>), grid, dim3(384), 0, s, L, qr, s1, tk, lnrho, S);
}

void launch_temp_sapply(const LevelDev& L, const double* S, const double* x, double* y, hipStream_t s) {
  vfill<double>(y, 0.0, L.n2, s);
  hipLaunchKernelGGL(k_temp_sapply, dim3((unsigned)(L.nmacro * L.ntiles)), dim3(384), 0, s, L, S, x, y);
}

void launch_mmoc(const LevelDev& L, const LocDev& loc, const double* F, const double* un, const double* uo, double tau,
                 double* out, hipStream_t s) {
  const long long tot = (long long)L.nloc2 * L.nmacro;
  hipLaunchKernelGGL(k_mmoc, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, L, loc, F, un, uo, tau, out);
}

void launch_scalar_dirichlet(const uint32_t* node, const uint8_t* kind, int nb, double* v, int set, double vin,
                             double vout, hipStream_t s) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_scalar_dirichlet, dim3((nb + 255) / 256), dim3(256), 0, s, node, kind, nb, v, set, vin, vout);
}
template void launch_vmass<float>(const LevelDev&, const VmassRule&, const float*, float, const float*, float*, bool,
                                  int, hipStream_t);

#define INST_V(R)                                                                  \
  template void vfill<R>(R*, R, long long, hipStream_t);                           \
  template void vcopy<R>(const R*, R*, long long, hipStream_t);                    \
  template void vaxpy<R>(R, const R*, R*, long long, hipStream_t);                 \
  template void vaxpby<R>(R, const R*, R, R*, long long, hipStream_t);             \
  template void vscale<R>(R, R*, long long, hipStream_t);                          \
  template void vmul<R>(const R*, const R*, R*, long long, hipStream_t);           \
  template void vinvert<R>(const R*, R*, long long, hipStream_t);                  \
  template void vdot<R>(const R*, const R*, long long, double*, double*, hipStream_t);         \
  template void vaxpy2_nrm<R>(R, const R*, R*, R, const R*, R*, long long, double*, double*, hipStream_t); \
  template void vcheb_start<R>(const R*, const R*, const R*, R, R*, R*, long long, hipStream_t); \
  template void vcheb_one<R>(const R*, const R*, const R*, R, R*, bool, long long, hipStream_t); \
  template void vcheb_step<R>(const R*, const R*, R, R, R*, R*, R*, bool, long long, hipStream_t); \
  template void vcheb_last<R>(const R*, const R*, R, R, const R*, const R*, R*, bool, long long, hipStream_t); \
  template void vsub<R>(const R*, const R*, R*, long long, hipStream_t);
INST_V(double)
INST_V(float)
template void vconvert<double, float>(const double*, float*, long long, hipStream_t);
INST_CG(double)
INST_CG(float)
template void vconvert<float, double>(const float*, double*, long long, hipStream_t);

// ---- fixed scratch of the allocation-free A-apply ------------------------------
// The shared-node slots of one plane-sweep apply for callers that cannot
// allocate device memory.  Every GPU the library runs on holds one copy until
// the process ends.  In host code this name stands for the device symbol and
// is not an address: host code uses the per-device address that
// hipGetSymbolAddress returns (noalloc_scratch).
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

void* noalloc_scratch(int device) {
  if (device < 0 || device >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

}  // namespace stk
