// C ABI, context, and host-side solver orchestration (Sec. 5.2 of
// arXiv 2506.04157): Chebyshev smoother, geometric multigrid V-cycle, A-block
// CG, V-cycle BFBT Schur approximation, symmetric Uzawa block
// preconditioner and the outer FGMRES, all launching the HIP kernels of
// kernels.hip on the caller's stream.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "device.hpp"
#include "mesh.hpp"
#include "stokes.h"

using namespace stk;

namespace {

thread_local std::string g_err;

struct StkError : std::runtime_error {
  int code;
  StkError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(x)                                                                                   \
  do {                                                                                              \
    hipError_t e_ = (x);                                                                            \
    if (e_ != hipSuccess) throw StkError(STK_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)
#define REQUIRE(c, msg) \
  do {                  \
    if (!(c)) throw StkError(STK_EINVAL, msg); \
  } while (0)

template <class F>
int guard(F&& f) {
  try {
    f();
    return STK_OK;
  } catch (StkError& e) {
    g_err = e.what();
    return e.code;
  } catch (std::bad_alloc&) {
    g_err = "host allocation failed";
    return STK_ENOMEM;
  } catch (std::exception& e) {
    g_err = e.what();
    return STK_EINVAL;
  }
}

template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void alloc(size_t count) {
    if (n == count && p) return;
    release();
    if (count == 0) count = 1;
    if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      throw StkError(STK_ENOMEM, "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed");
    }
    n = count;
  }
  void upload(const std::vector<T>& v) {
    alloc(v.size());
    if (!v.empty()) HIPCHK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  }
};

// work vectors of one precision on one level
template <class R>
struct Pool {
  std::vector<std::unique_ptr<DBuf<R>>> v;
  R* get(size_t k, size_t count, hipStream_t s) {
    while (v.size() <= k) v.emplace_back(new DBuf<R>());
    if (v[k]->n != count || !v[k]->p) {
      v[k]->alloc(count);
      HIPCHK(hipMemsetAsync(v[k]->p, 0, count * sizeof(R), s));
    }
    return v[k]->p;
  }
};

struct LevelData {
  Level h;
  LevelDev d{};
  BcDev bc{};
  DBuf<uint32_t> l2g2, l2g1, dir, fs;
  DBuf<double> tinv, nrm, eta, dinv;
  DBuf<float> tinvf, nrmf, etaf, dinvf;
  DBuf<int> tiles;
  Sweep sw;
  DBuf<int> eall;
  DBuf<int> xt_tab, xt_off;   // grid-transfer table (this level coarse)
  DBuf<int> sw_strip, sw_plist2, sw_poff2, sw_plist1, sw_poff1, sw_elist, sw_eoff, sw_etab, g2ptr, g2slot, g1ptr, g1slot;
  DBuf<uint32_t> g2node, g1node, sw_g2tab, sw_g1tab;
  DBuf<double> sl2_64, sl1_64;   // slot buffers of the sweep kernels
  DBuf<float> sl2_32, sl1_32;
  // P1 mass stencil: lattice tables, gather lists, coefficients, slots
  DBuf<int16_t> ms_nb;
  DBuf<int> ms_dst, ms_incptr, ms_inc, ms_gptr, ms_gslot;
  DBuf<uint32_t> ms_gnode;
  DBuf<double> ms_c64, ms_sl64;
  DBuf<float> ms_c32, ms_sl32;
  template <class R> R* msl();
  double lo = 0, hi = 0;
  bool bounds_set = false;
  Pool<double> p64, q64;   // velocity-size / pressure-size work vectors
  Pool<float> p32, q32;
  template <class R> Pool<R>& pool();
  template <class R> Pool<R>& ppool();
  template <class R> const R* etap() const;
  template <class R> const R* dinvp() const;
  template <class R> R* sl2();
  template <class R> R* sl1();
  // P1 Poisson stencils K_{1/sqrt eta} of the weighted BFBT (eq. schurWBFBT)
  // for up to two element factors a^2, with their inverse diagonals
  struct PoissonSet {
    double a2 = -1.0;
    int gen = -1;
    DBuf<double> c64, dinv64;
    DBuf<float> c32, dinv32;
    template <class R> const R* coef() const;
    template <class R> const R* dinv() const;
  };
  PoissonSet ps[2];
  // P2 temperature of the level (quadrature-point viscosity)
  DBuf<double> T2;
  DBuf<float> T2f;
  // coarsest level: element matrices and node data of its CG
  bool ccg = false;   // set on the coarsest level
  CoarseDev cd{};
  DBuf<uint32_t> c_enode;
  DBuf<double> c_emat, c_nrm;
  DBuf<float> c_ematf;
  DBuf<int> c_iptr, c_pos;
  DBuf<uint8_t> c_act;
};
template <> const double* LevelData::PoissonSet::coef<double>() const { return c64.p; }
template <> const float* LevelData::PoissonSet::coef<float>() const { return c32.p; }
template <> const double* LevelData::PoissonSet::dinv<double>() const { return dinv64.p; }
template <> const float* LevelData::PoissonSet::dinv<float>() const { return dinv32.p; }
template <> Pool<double>& LevelData::pool<double>() { return p64; }
template <> Pool<float>& LevelData::pool<float>() { return p32; }
template <> Pool<double>& LevelData::ppool<double>() { return q64; }
template <> Pool<float>& LevelData::ppool<float>() { return q32; }
template <> const double* LevelData::etap<double>() const { return eta.p; }
template <> const float* LevelData::etap<float>() const { return etaf.p; }
template <> const double* LevelData::dinvp<double>() const { return dinv.p; }
template <> const float* LevelData::dinvp<float>() const { return dinvf.p; }
template <> double* LevelData::sl2<double>() {
  sl2_64.alloc((size_t)3 * d.nmacro * sw.nsh2);
  return sl2_64.p;
}
template <> float* LevelData::sl2<float>() {
  sl2_32.alloc((size_t)3 * d.nmacro * sw.nsh2);
  return sl2_32.p;
}
template <> double* LevelData::sl1<double>() {
  sl1_64.alloc((size_t)d.nmacro * sw.nsh1);
  return sl1_64.p;
}
template <> float* LevelData::sl1<float>() {
  sl1_32.alloc((size_t)d.nmacro * sw.nsh1);
  return sl1_32.p;
}

template <> double* LevelData::msl<double>() {
  ms_sl64.alloc((size_t)d.nmacro * d.ms.nsh);
  return ms_sl64.p;
}
template <> float* LevelData::msl<float>() {
  ms_sl32.alloc((size_t)d.nmacro * d.ms.nsh);
  return ms_sl32.p;
}

// indices into the per-level velocity work pools
enum { W_B = 0, W_X, W_R, W_D, W_T, W_CG_R, W_CG_Z, W_CG_P, W_CG_Q, W_U0, W_U1, W_U2, W_U3, W_U4, W_U5,
       W_VM_R, W_VM_Z, W_VM_P, W_VM_Q, W_VM_T, W_VM_Z2,
       W_F0, W_F1, W_F2, W_F3, W_C_R, W_C_Z, W_C_P, W_C_Q, W_C_B, W_C_X, W_PC0, W_PC1, W_C_Y };
// pressure-size pools
enum { Q_0 = 0, Q_1, Q_2, Q_3, Q_4, Q_5, Q_6, Q_7, Q_8, Q_9, Q_ONES, Q_MD, Q_U0, Q_U1, Q_F0, Q_F1, Q_F2, Q_F3,
       Q_P1T, Q_P1R, Q_P1B, Q_P1X, Q_P1C_R, Q_P1C_Z, Q_P1C_P, Q_P1C_Q, Q_PK_R, Q_PK_Z, Q_PK_P, Q_PK_Q, Q_WB1, Q_WB2 };

}  // namespace

struct stk_ctx {
  stk_mesh_desc desc{};
  int device = 0;          // HIP device current at stk_create
  MacroMesh mm;
  Topology top;
  std::vector<std::unique_ptr<LevelData>> lv;   // index = level; [0, min_level) unused
  DBuf<double> geo;
  DBuf<float> geof;
  DBuf<uint8_t> bact, own;
  hipStream_t s = nullptr;
  DBuf<double> dotbuf;
  DBuf<double> cgbuf;      // device CG scalars
  DBuf<double> cgpart;     // device CG partial sums
  double* hpin = nullptr;
  double* hcg = nullptr;         // two pinned copies of the device CG scalars
  hipEvent_t cgev[2] = {nullptr, nullptr};
  bool ready = false;
  bool has_rho = false;
  // weighted BFBT: the vector mass rule, the field generation the cached
  // operators belong to, and the inverse diagonals of the vector masses
  VmassRule vrule{};
  int field_gen = 0;
  struct VmassDiag {
    double a2 = -1.0;
    int gen = -1;
    DBuf<double> d64;
    DBuf<float> d32;
  } vmd[2];
  // free slip on both spheres: the rigid rotations are removed from the
  // finest-level velocities the solvers work with
  bool rot = false;
  DBuf<double> rotX, rotbuf;
  DBuf<double> meanbuf;    // partial sums of the device-side mean removal
  RotDev rotd{};
  // temperature step: Dirichlet node list of the finest level, the point
  // locator of the MMOC, work vectors and FGMRES storage
  struct TempData {
    bool ready = false;
    DBuf<uint32_t> bnode;
    DBuf<uint8_t> bkind;
    int nb = 0;
    DBuf<int> prism;
    DBuf<double> minv;
    LocDev loc{};
    DBuf<double> w, fg;
    DBuf<double> smat;     // stored element matrices of S (STK_TEMP_SYM_STORED, stored_S)
    DBuf<double> tstar, fbuf;   // stk_coupled_step: extrapolated temperature, buoyancy
  } temp;
  DBuf<double> lnrho;
  DBuf<float> lnrhof;
  DBuf<double> vbase;      // radial base viscosity samples (quadrature-point viscosity)
  stk_solver_params par{};
  stk_report* rep = nullptr;
  // FGMRES storage
  DBuf<double> fg;
  // stk_kernel_timer: event pairs around the finest-level A sweeps
  bool timer_on = false;
  int timer_n = 0;
  std::vector<hipEvent_t> timer_ev;
  bool verbose = std::getenv("STK_VERBOSE") != nullptr;   // progress lines on stderr
  int L() const { return desc.level; }
  int lmin() const { return desc.min_level; }
  LevelData& at(int l) { return *lv[l]; }
  template <class R> const R* rho() const;
};
template <> const double* stk_ctx::rho<double>() const { return has_rho ? lnrho.p : nullptr; }
template <> const float* stk_ctx::rho<float>() const { return has_rho ? lnrhof.p : nullptr; }

namespace {

using Ctx = stk_ctx;

long long n2of(Ctx& c, int l) { return c.at(l).h.n2; }
long long n1of(Ctx& c, int l) { return c.at(l).h.n1; }

template <class R>
double dot(Ctx& c, const R* x, const R* y, long long n) {
  vdot<R>(x, y, n, c.dotbuf.p, c.dotbuf.p + 2 * DOT_BLOCKS, c.s);
  HIPCHK(hipMemcpyAsync(c.hpin, c.dotbuf.p + 2 * DOT_BLOCKS, sizeof(double), hipMemcpyDeviceToHost, c.s));
  HIPCHK(hipStreamSynchronize(c.s));
  return *c.hpin;
}
template <class R>
double nrm2(Ctx& c, const R* x, long long n) { return std::sqrt(dot<R>(c, x, x, n)); }
// CG update x += alpha p, r -= alpha q; returns |r| of the updated r
template <class R>
double cg_step_nrm(Ctx& c, double alpha, const R* p, R* x, const R* q, R* r, long long n) {
  vaxpy2_nrm<R>(R(alpha), p, x, R(-alpha), q, r, n, c.dotbuf.p, c.dotbuf.p + 2 * DOT_BLOCKS, c.s);
  HIPCHK(hipMemcpyAsync(c.hpin, c.dotbuf.p + 2 * DOT_BLOCKS, sizeof(double), hipMemcpyDeviceToHost, c.s));
  HIPCHK(hipStreamSynchronize(c.s));
  return std::sqrt(*c.hpin);
}

// P_v (Dirichlet -> 0, free slip -> tangential); on the finest level with
// free slip on both spheres also the removal of the rigid rotations
template <class R>
void rot_remove(Ctx& c, R* v) {
  launch_rot_remove<R>(c.rotd, n2of(c, c.L()), v, c.rotbuf.p, c.s);
}
template <class R>
void project(Ctx& c, int l, R* v) {
  launch_project<R>(c.at(l).bc, n2of(c, l), v, c.s);
  if (c.rot && l == c.L()) rot_remove<R>(c, v);
}

template <class R>
R* ones(Ctx& c) {
  LevelData& F = c.at(c.L());
  Pool<R>& q = F.ppool<R>();
  bool fresh = q.v.size() <= Q_ONES || !q.v[Q_ONES]->p;
  R* o = q.get(Q_ONES, n1of(c, c.L()), c.s);
  if (fresh) vfill<R>(o, R(1), n1of(c, c.L()), c.s);
  return o;
}

// P_p: arithmetic mean zero (Sec. 5.1)
template <class R>
void project_mean(Ctx& c, R* p) {
  const long long n1 = n1of(c, c.L());
  double mean = dot<R>(c, p, ones<R>(c), n1) / (double)n1;
  vaxpy<R>(R(-mean), ones<R>(c), p, n1, c.s);
}

// ---- operator applies (outputs overwritten) ---------------------------------
template <class R>
void sweep(Ctx& c, int l, int flags, const R* u, const R* p, const R* eta, const R* rho, R* yu, R* yp, int bc) {
  LevelData& L = c.at(l);
  launch_stokes<R>(flags, L.d, L.bc, u, p, eta, rho, yu, yp, L.sl2<R>(), L.sl1<R>(), bc, c.s);
}
constexpr int TIMER_MAX = 4096;
template <class R>
void applyA(Ctx& c, int l, const R* x, R* y, int bc) {
  LevelData& L = c.at(l);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c.timer_on && l == c.L() && !L.d.elemwise && c.timer_n < TIMER_MAX) {
    while ((int)c.timer_ev.size() < 2 * (c.timer_n + 1)) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      c.timer_ev.push_back(e);
    }
    e0 = c.timer_ev[2 * c.timer_n];
    e1 = c.timer_ev[2 * c.timer_n + 1];
    ++c.timer_n;
  }
  launch_stokes<R>(F_A, L.d, L.bc, x, nullptr, L.etap<R>(), nullptr, y, nullptr, L.sl2<R>(), L.sl1<R>(), bc, c.s,
                   e0, e1);
}
template <class R>
void applyB(Ctx& c, int l, const R* u, R* q, bool withC, int bc) {
  REQUIRE(!withC || (c.has_rho && l == c.L()), "C block needs ln rho on the finest level");
  sweep<R>(c, l, withC ? (F_B | F_C) : F_B, u, nullptr, nullptr, c.rho<R>(), nullptr, q, bc);
}
template <class R>
void applyBt(Ctx& c, int l, const R* p, R* y, bool withCt, int bc) {
  REQUIRE(!withCt || (c.has_rho && l == c.L()), "C block needs ln rho on the finest level");
  sweep<R>(c, l, withCt ? (F_BT | F_CT) : F_BT, nullptr, p, nullptr, c.rho<R>(), y, nullptr, bc);
}
template <class R>
void applyMass(Ctx& c, int l, const R* p, R* q) {
  LevelData& L = c.at(l);
  if (L.d.ms.on) launch_mass_stencil<R>(L.d, p, q, L.msl<R>(), c.s);
  else sweep<R>(c, l, F_M, nullptr, p, L.etap<R>(), nullptr, nullptr, q, 0);
}
// K [u;p] on the finest level, velocity projected on both sides
template <class R>
void applyK(Ctx& c, const R* u, const R* p, R* yu, R* yp, bool transpose, int bc) {
  const int l = c.L();
  int fl = F_A | F_BT | F_B;
  if (c.has_rho) fl |= transpose ? F_CT : F_C;
  sweep<R>(c, l, fl, u, p, c.at(l).etap<R>(), c.rho<R>(), yu, yp, bc);
}

// ---- Chebyshev smoother (Jacobi preconditioned) -------------------------------
template <class R>
void chebyshev(Ctx& c, int l, const R* b, R* x, int steps, int deg, bool xzero) {
  LevelData& L = c.at(l);
  const long long N = 3 * L.h.n2;
  const double theta = 0.5 * (L.hi + L.lo), delta = 0.5 * (L.hi - L.lo), sigma = theta / delta;
  R* r = L.pool<R>().get(W_R, N, c.s);
  R* d = L.pool<R>().get(W_D, N, c.s);
  R* t = L.pool<R>().get(W_T, N, c.s);
  const R* dinv = L.dinvp<R>();
  for (int st = 0; st < steps; ++st) {
    // r = b - A x (b and A's output are projected).  The directions d stay
    // unprojected: A projects its input, and since the projection is linear
    // and x enters projected, projecting x after the step leaves exactly the
    // sum of the projected directions.
    const bool x0 = xzero && st == 0;   // x enters as zero
    if (!x0) applyA<R>(c, l, x, t, BCM_IN | BCM_OUT);
    if (deg == 1) {
      vcheb_one<R>(b, x0 ? nullptr : t, dinv, R(1.0 / theta), x, !x0, N, c.s);
    } else {
      vcheb_start<R>(b, x0 ? nullptr : t, dinv, R(1.0 / theta), r, d, N, c.s);
      double rho_old = 1.0 / sigma;
      for (int k = 1; k < deg; ++k) {
        // x += d; r -= A d; d = 2 rho/delta D^-1 r + rho rho_old d (the last
        // direction goes into x at once)
        applyA<R>(c, l, d, t, BCM_IN | BCM_OUT);
        const double rho = 1.0 / (2.0 * sigma - rho_old);
        const bool xin = !(x0 && k == 1);
        if (k + 1 < deg)
          vcheb_step<R>(t, dinv, R(2.0 * rho / delta), R(rho * rho_old), r, x, d, xin, N, c.s);
        else
          vcheb_last<R>(t, dinv, R(2.0 * rho / delta), R(rho * rho_old), r, d, x, xin, N, c.s);
        rho_old = rho;
      }
    }
    project<R>(c, l, x);
  }
}

// ---- coarse grid: Jacobi-preconditioned CG in FP64 (Sec. 5.2.2, tol_coarse) ---
// Drives a device-resident CG: step(it) enqueues iteration it; chunks of
// `chunk` iterations are enqueued one ahead of the host's look at the device
// scalars (convergence flag, iteration count) of the chunk before, so the
// GPU never waits for the host.  Kernels of a finished solve return at once,
// so the chunk in flight when the flag is seen costs only its launches.
// Returns the device's iteration count.
template <class Step>
int run_chunks(Ctx& c, const double* sc, int chunk, int maxit, Step step) {
  int it = 0, k = 0;
  for (;;) {
    for (int i = 0; i < chunk && it < maxit; ++i, ++it) step(it);
    const int cur = k & 1;
    HIPCHK(hipMemcpyAsync(c.hcg + cur * CGS_N, sc, CGS_N * sizeof(double), hipMemcpyDeviceToHost, c.s));
    HIPCHK(hipEventRecord(c.cgev[cur], c.s));
    ++k;
    if (k >= 2) {
      const double* h = c.hcg + (cur ^ 1) * CGS_N;
      HIPCHK(hipEventSynchronize(c.cgev[cur ^ 1]));
      if (h[CGS_DONE] != 0.0) return (int)h[CGS_IT];
    }
    if (it >= maxit) break;
  }
  HIPCHK(hipEventSynchronize(c.cgev[(k - 1) & 1]));
  return (int)c.hcg[((k - 1) & 1) * CGS_N + CGS_IT];
}

// Jacobi-preconditioned CG with device-resident scalars (no host round trip
// per iteration; see run_chunks).  apply(p, q) computes q = A p; proj(v)
// projects in place (it must be an orthogonal projection commuting with the
// residual's range).
template <class R, class Apply, class Proj>
int dev_pcg(Ctx& c, long long N, Apply apply, Proj proj, const R* dinv, const R* b, R* x, R* r, R* z, R* p, R* q,
            double tol, int maxit, int chunk) {
  double* part = c.cgpart.p;
  double* sc = c.cgbuf.p;
  vfill<R>(x, R(0), N, c.s);
  vcopy<R>(b, r, N, c.s);
  proj(r);
  cg_init<R>(r, dinv, z, N, tol, part, sc, c.s);
  proj(z);
  vcopy<R>(z, p, N, c.s);
  return run_chunks(c, sc, chunk, maxit, [&](int it) {
    const int parity = it & 1;
    apply(p, q);
    cg_dot<R>(p, q, N, part, sc, c.s);
    cg_update<R>(p, q, dinv, x, r, z, N, part, sc, parity, c.s);
    proj(z);
    cg_pupdate<R>(z, p, N, part, sc, parity, c.s);
  });
}

// fp32: the FP32 preconditioner's coarse solve (element matrices rounded to
// FP32; vectors, scalars and accumulation stay FP64)
void coarse_cg64(Ctx& c, const double* b, double* x, double tol, int maxit, bool fp32) {
  const int l = c.lmin();
  LevelData& L = c.at(l);
  const long long N = 3 * L.h.n2;
  Pool<double>& P = L.pool<double>();
  double* r = P.get(W_C_R, N, c.s);
  double* z = P.get(W_C_Z, N, c.s);
  double* p = P.get(W_C_P, N, c.s);
  double* q = P.get(W_C_Q, N, c.s);
  double* Y = P.get(W_C_Y, (size_t)L.cd.ne * 30, c.s);
  double* part = c.cgpart.p;
  double* sc = c.cgbuf.p;
  ccg_init(L.cd, b, x, r, z, tol, part, sc, c.s);
  const int its = run_chunks(c, sc, 4, maxit,
                             [&](int it) { ccg_iter(L.cd, fp32, x, r, z, p, q, Y, part, sc, it, c.s); });
  if (c.rep) c.rep->coarse_its += its;
}

template <class R>
void coarse_solve(Ctx& c, const R* b, R* x) {
  const int l = c.lmin();
  LevelData& L = c.at(l);
  const long long N = 3 * L.h.n2;
  if (std::is_same<R, double>::value) {
    coarse_cg64(c, (const double*)b, (double*)x, c.par.tol_coarse, c.par.max_inner * 10, false);
  } else {
    double* b64 = L.pool<double>().get(W_C_B, N, c.s);
    double* x64 = L.pool<double>().get(W_C_X, N, c.s);
    vconvert<float, double>((const float*)b, b64, N, c.s);
    coarse_cg64(c, b64, x64, c.par.tol_coarse, c.par.max_inner * 10, true);
    vconvert<double, float>(x64, (float*)x, N, c.s);
  }
}

// ---- V-cycle (Sec. 5.2.2, Fig. ASolverStructure) ------------------------------
template <class R>
void vcycle(Ctx& c, int l, const R* b, R* x, int steps, int deg) {
  if (l == c.lmin()) {
    coarse_solve<R>(c, b, x);
    return;
  }
  LevelData& L = c.at(l);
  LevelData& C = c.at(l - 1);
  const long long N = 3 * L.h.n2, Nc = 3 * C.h.n2;
  chebyshev<R>(c, l, b, x, steps, deg, true);   // writes x without reading it
  R* t = L.pool<R>().get(W_T, N, c.s);
  applyA<R>(c, l, x, t, BCM_IN | BCM_OUT);
  R* bc = C.pool<R>().get(W_B, Nc, c.s);
  R* xc = C.pool<R>().get(W_X, Nc, c.s);
  vfill<R>(bc, R(0), Nc, c.s);
  launch_restrict_diff<R>(C.d, L.d, b, t, bc, BCM_IN | BCM_OUT, c.s);   // R (b - A x)
  vcycle<R>(c, l - 1, bc, xc, steps, deg);
  launch_prolong_add<R>(C.d, L.d, xc, x, BCM_OUT, c.s);                 // x += P x_c
  chebyshev<R>(c, l, b, x, steps, deg, false);
  if (c.rep) c.rep->vcycles += (l == c.L());
}

// ---- A-block solve: CG preconditioned by one V-cycle (Sec. 5.2.2, tol_A) -------
template <class R>
void solve_A(Ctx& c, const R* b, R* x) {
  const int l = c.L();
  LevelData& L = c.at(l);
  const long long N = 3 * L.h.n2;
  Pool<R>& P = L.pool<R>();
  R* r = P.get(W_CG_R, N, c.s);
  R* z = P.get(W_CG_Z, N, c.s);
  R* p = P.get(W_CG_P, N, c.s);
  R* q = P.get(W_CG_Q, N, c.s);
  vfill<R>(x, R(0), N, c.s);
  vcopy<R>(b, r, N, c.s);
  project<R>(c, l, r);
  const double nb = nrm2<R>(c, r, N);
  if (c.rep) c.rep->a_solves++;
  if (nb == 0.0) return;
  vcycle<R>(c, l, r, z, c.par.m_A, c.par.deg_A);
  vcopy<R>(z, p, N, c.s);
  double rz = dot<R>(c, r, z, N);
  for (int it = 1; it <= c.par.max_inner; ++it) {
    if (c.rep) c.rep->a_cg_its++;
    applyA<R>(c, l, p, q, BCM_IN | BCM_OUT);
    if (c.rot) rot_remove<R>(c, q);
    const double alpha = rz / dot<R>(c, p, q, N);
    if (cg_step_nrm<R>(c, alpha, p, x, q, r, N) <= c.par.tol_A * nb) break;
    vcycle<R>(c, l, r, z, c.par.m_A, c.par.deg_A);
    const double rz2 = dot<R>(c, r, z, N);
    vaxpby<R>(R(1), z, R(rz2 / rz), p, N, c.s);
    rz = rz2;
  }
}

// ---- M_{1/eta} solve: Jacobi CG to tol_invmass (Sec. 5.2.3) --------------------
template <class R>
void solve_mass(Ctx& c, const R* b, R* x) {
  const int l = c.L();
  LevelData& L = c.at(l);
  const long long n1 = L.h.n1;
  Pool<R>& Q = L.ppool<R>();
  R* md = Q.get(Q_MD, n1, c.s);   // inverse diagonal, filled by set_fields
  R* r = Q.get(Q_6, n1, c.s);
  R* p = Q.get(Q_7, n1, c.s);
  R* q = Q.get(Q_8, n1, c.s);
  R* z = Q.get(Q_9, n1, c.s);
  const int its = dev_pcg<R>(
      c, n1, [&](const R* pp, R* qq) { applyMass<R>(c, l, pp, qq); }, [](R*) {}, md, b, x, r, z, p, q,
      c.par.tol_invmass, c.par.max_inner * 10, n1 > 1000000 ? 1 : 4);
  if (c.rep) c.rep->mass_its += its;
}

// The BFBT inner operator C^-1 of the chosen Schur approximation: one V-cycle
// Ac (m_V, deg_V) for the V-cycle BFBT (eq. schurV), diag(A)^-1 (projected)
// for the diag(A)-BFBT (Sec. 5.2.3)
template <class R>
void bfbt_cinv(Ctx& c, const R* in, R* out) {
  const int l = c.L();
  LevelData& L = c.at(l);
  const long long N = 3 * L.h.n2;
  if (c.par.schur == STK_SCHUR_DIAG_BFBT) {
    vmul<R>(L.dinvp<R>(), in, out, N, c.s);
    project<R>(c, l, out);
  } else {
    vcycle<R>(c, l, in, out, c.par.m_V, c.par.deg_V);
  }
}

// S_C p = B C^-1 B^T p
template <class R>
void apply_SC(Ctx& c, const R* p, R* y) {
  const int l = c.L();
  LevelData& L = c.at(l);
  const long long N = 3 * L.h.n2;
  R* t = L.pool<R>().get(W_U3, N, c.s);
  R* z = L.pool<R>().get(W_U4, N, c.s);
  applyBt<R>(c, l, p, t, false, BCM_OUT);
  bfbt_cinv<R>(c, t, z);
  applyB<R>(c, l, z, y, false, BCM_IN);
  project_mean<R>(c, y);
}

// CG on S_C preconditioned by M_{1/eta}^-1, to tol_vbfbt (Sec. 5.2.3)
template <class R>
void solve_SC(Ctx& c, const R* b, R* x) {
  const int l = c.L();
  LevelData& L = c.at(l);
  const long long n1 = L.h.n1;
  Pool<R>& Q = L.ppool<R>();
  R* r = Q.get(Q_2, n1, c.s);
  R* z = Q.get(Q_3, n1, c.s);
  R* p = Q.get(Q_4, n1, c.s);
  R* q = Q.get(Q_5, n1, c.s);
  vfill<R>(x, R(0), n1, c.s);
  vcopy<R>(b, r, n1, c.s);
  project_mean<R>(c, r);
  const double nb = nrm2<R>(c, r, n1);
  if (c.rep) c.rep->s_solves++;
  if (nb == 0.0) return;
  solve_mass<R>(c, r, z);
  project_mean<R>(c, z);
  vcopy<R>(z, p, n1, c.s);
  double rz = dot<R>(c, r, z, n1);
  for (int it = 1; it <= c.par.max_inner; ++it) {
    if (c.rep) c.rep->s_cg_its++;
    apply_SC<R>(c, p, q);
    const double alpha = rz / dot<R>(c, p, q, n1);
    if (cg_step_nrm<R>(c, alpha, p, x, q, r, n1) <= c.par.tol_vbfbt * nb) break;
    solve_mass<R>(c, r, z);
    project_mean<R>(c, z);
    const double rz2 = dot<R>(c, r, z, n1);
    vaxpby<R>(R(1), z, R(rz2 / rz), p, n1, c.s);
    rz = rz2;
  }
}

// V-cycle BFBT, eq. (schurV): (B Ac^-1 B^T)^-1 (B Ac^-1 A Ac^-1 B^T) (B Ac^-1 B^T)^-1
template <class R>
void schur_vbfbt(Ctx& c, const R* rp, R* out) {
  const int l = c.L();
  LevelData& L = c.at(l);
  const long long N = 3 * L.h.n2, n1 = L.h.n1;
  Pool<R>& Q = L.ppool<R>();
  R* y1 = Q.get(Q_0, n1, c.s);
  R* y2 = Q.get(Q_1, n1, c.s);
  R* t = L.pool<R>().get(W_U3, N, c.s);
  R* z = L.pool<R>().get(W_U4, N, c.s);
  R* w = L.pool<R>().get(W_U5, N, c.s);
  solve_SC<R>(c, rp, y1);
  applyBt<R>(c, l, y1, t, false, BCM_OUT);
  bfbt_cinv<R>(c, t, z);
  applyA<R>(c, l, z, w, BCM_IN | BCM_OUT);
  bfbt_cinv<R>(c, w, z);
  applyB<R>(c, l, z, y2, false, BCM_IN);
  project_mean<R>(c, y2);
  solve_SC<R>(c, y2, out);
}

// ---- weighted BFBT (Sec. 5.2.3, eq. schurWBFBT) -----------------------------------
// The P1 Poisson stencil K_{1/sqrt eta} of level l for the element factor a2
// (built for the current fields on first use; two factors per level kept).
LevelData::PoissonSet& poisson_set(Ctx& c, int l, double a2) {
  LevelData& L = c.at(l);
  for (auto& p : L.ps)
    if (p.a2 == a2 && p.gen == c.field_gen) return p;
  REQUIRE(L.d.ms.on, "the P1 stencil layout is not available on this level");
  LevelData::PoissonSet& P = L.ps[0].gen != c.field_gen ? L.ps[0] : L.ps[1];
  const size_t nc = (size_t)L.d.nmacro * NSTORE1 * (L.h.nloc1 + 1);
  P.c64.alloc(nc);
  P.c32.alloc(nc);
  P.dinv64.alloc(L.h.n1);
  P.dinv32.alloc(L.h.n1);
  launch_poisson_stencil_build(L.d, L.eta.p, a2, P.c64.p, P.c32.p, c.s);
  launch_stencil_diag<double>(L.d, P.c64.p, P.dinv64.p, c.s);
  vinvert<double>(P.dinv64.p, P.dinv64.p, L.h.n1, c.s);
  vconvert<double, float>(P.dinv64.p, P.dinv32.p, L.h.n1, c.s);
  P.a2 = a2;
  P.gen = c.field_gen;
  return P;
}

template <class R>
void apply_poisson(Ctx& c, int l, const LevelData::PoissonSet& P, const R* p, R* q) {
  LevelData& L = c.at(l);
  launch_stencil<R>(L.d, P.coef<R>(), p, q, L.msl<R>(), c.s);
}

// Multigrid V-cycle for the Poisson problem on nested P1 spaces: damped Jacobi
// smoothing (WB_SMOOTH sweeps before and after, weight WB_OMEGA), restriction
// P^T, coarse Jacobi-CG to WB_COARSE_TOL, prolongation P; x overwritten.  The
// Neumann operator is singular with the constants as kernel; a right-hand side
// of zero sum stays so under P^T (the rows of P sum to one), so the coarse
// problems are consistent.
constexpr int WB_SMOOTH = 2;
constexpr double WB_OMEGA = 0.6;
// coarse CG tolerance: the Neumann problem is consistent only up to the
// rounding of the restriction, so FP32 stops well above its unit roundoff
template <class R> constexpr double wb_coarse_tol() { return sizeof(R) == 8 ? 1e-10 : 1e-5; }
template <class R>
void vcycle_p1(Ctx& c, int l, double a2, const R* b, R* x) {
  LevelData& L = c.at(l);
  const long long n1 = L.h.n1;
  const LevelData::PoissonSet& P = poisson_set(c, l, a2);
  Pool<R>& Q = L.ppool<R>();
  auto K = [&](const R* v, R* y) { apply_poisson<R>(c, l, P, v, y); };
  if (l == c.lmin()) {
    R* r = Q.get(Q_P1C_R, n1, c.s);
    R* z = Q.get(Q_P1C_Z, n1, c.s);
    R* p = Q.get(Q_P1C_P, n1, c.s);
    R* q = Q.get(Q_P1C_Q, n1, c.s);
    const int its = dev_pcg<R>(
        c, n1, K, [&](R* v) { launch_remove_mean<R>(v, n1, c.meanbuf.p, c.s); }, P.dinv<R>(), b, x, r, z, p, q,
        wb_coarse_tol<R>(), c.par.max_inner * 10, 4);
    if (c.rep) c.rep->coarse_its += its;
    return;
  }
  LevelData& C = c.at(l - 1);
  R* t = Q.get(Q_P1T, n1, c.s);
  R* r = Q.get(Q_P1R, n1, c.s);
  R* bc = C.ppool<R>().get(Q_P1B, C.h.n1, c.s);
  R* xc = C.ppool<R>().get(Q_P1X, C.h.n1, c.s);
  const R* dinv = P.dinv<R>();
  vcheb_one<R>(b, nullptr, dinv, R(WB_OMEGA), x, false, n1, c.s);   // x = w D^-1 b
  for (int k = 1; k < WB_SMOOTH; ++k) {
    K(x, t);
    vcheb_one<R>(b, t, dinv, R(WB_OMEGA), x, true, n1, c.s);        // x += w D^-1 (b - K x)
  }
  K(x, t);
  vsub<R>(b, t, r, n1, c.s);
  launch_p1_restrict<R>(C.d, L.d, r, bc, c.s);
  vcycle_p1<R>(c, l - 1, a2, bc, xc);
  launch_p1_prolong<R>(C.d, L.d, xc, t, c.s);
  vaxpy<R>(R(1), t, x, n1, c.s);
  for (int k = 0; k < WB_SMOOTH; ++k) {
    K(x, t);
    vcheb_one<R>(b, t, dinv, R(WB_OMEGA), x, true, n1, c.s);
  }
}

// K_{1/sqrt eta}^-1 b on the finest level: CG preconditioned by the P1
// V-cycle, stopped at |r| <= tol_wbfbt |r0| or |r| <= tol_wbfbt (whichever
// comes first, Table parametertable); b and x of arithmetic mean zero.
template <class R>
void solve_poisson(Ctx& c, double a2, const R* b, R* x) {
  const int l = c.L();
  LevelData& L = c.at(l);
  const long long n1 = L.h.n1;
  const LevelData::PoissonSet& P = poisson_set(c, l, a2);
  Pool<R>& Q = L.ppool<R>();
  R* r = Q.get(Q_PK_R, n1, c.s);
  R* z = Q.get(Q_PK_Z, n1, c.s);
  R* p = Q.get(Q_PK_P, n1, c.s);
  R* q = Q.get(Q_PK_Q, n1, c.s);
  vfill<R>(x, R(0), n1, c.s);
  vcopy<R>(b, r, n1, c.s);
  project_mean<R>(c, r);
  const double nb = nrm2<R>(c, r, n1);
  if (c.rep) c.rep->s_solves++;
  if (nb == 0.0) return;
  const double stop = std::max(c.par.tol_wbfbt * nb, c.par.tol_wbfbt);
  vcycle_p1<R>(c, l, a2, r, z);
  project_mean<R>(c, z);
  vcopy<R>(z, p, n1, c.s);
  double rz = dot<R>(c, r, z, n1);
  for (int it = 1; it <= c.par.max_inner * 10; ++it) {
    if (c.rep) c.rep->s_cg_its++;
    apply_poisson<R>(c, l, P, p, q);
    const double alpha = rz / dot<R>(c, p, q, n1);
    cg_step_nrm<R>(c, alpha, p, x, q, r, n1);
    // K p sums to zero only up to rounding: keep r free of the constant, or
    // the recurrence stalls at the rounding level (FP32)
    launch_remove_mean<R>(r, n1, c.meanbuf.p, c.s);
    if (nrm2<R>(c, r, n1) <= stop) break;
    vcycle_p1<R>(c, l, a2, r, z);
    project_mean<R>(c, z);
    const double rz2 = dot<R>(c, r, z, n1);
    vaxpby<R>(R(1), z, R(rz2 / rz), p, n1, c.s);
    rz = rz2;
  }
  project_mean<R>(c, x);
}

// The inverse diagonal of the vector mass M_{sqrt eta} for the factor a2
Ctx::VmassDiag& vmass_diag(Ctx& c, double a2) {
  for (auto& d : c.vmd)
    if (d.a2 == a2 && d.gen == c.field_gen) return d;
  Ctx::VmassDiag& D = c.vmd[0].gen != c.field_gen ? c.vmd[0] : c.vmd[1];
  LevelData& L = c.at(c.L());
  const long long N = 3 * L.h.n2;
  D.d64.alloc(N);
  D.d32.alloc(N);
  launch_vmass<double>(L.d, c.vrule, L.eta.p, a2, nullptr, D.d64.p, true, 0, c.s);
  vinvert<double>(D.d64.p, D.d64.p, N, c.s);
  vconvert<double, float>(D.d64.p, D.d32.p, N, c.s);
  D.a2 = a2;
  D.gen = c.field_gen;
  return D;
}

// y = P M_{sqrt eta} P u on the finest level
template <class R>
void apply_vmass(Ctx& c, double a2, const R* u, R* y) {
  LevelData& L = c.at(c.L());
  launch_vmass<R>(L.d, c.vrule, L.etap<R>(), R(a2), u, y, false, BCM_IN, c.s);
  project<R>(c, c.L(), y);
}

// M_{sqrt eta}^-1 b on the admissible velocities: Jacobi-CG to tol_vmass
template <class R>
void solve_vmass(Ctx& c, double a2, const R* b, R* x) {
  const int l = c.L();
  LevelData& L = c.at(l);
  const long long N = 3 * L.h.n2;
  Ctx::VmassDiag& D = vmass_diag(c, a2);
  const R* dinv = std::is_same<R, double>::value ? (const R*)D.d64.p : (const R*)D.d32.p;
  Pool<R>& P = L.pool<R>();
  R* r = P.get(W_VM_R, N, c.s);
  R* z = P.get(W_VM_Z, N, c.s);
  R* p = P.get(W_VM_P, N, c.s);
  R* q = P.get(W_VM_Q, N, c.s);
  const int its = dev_pcg<R>(
      c, N, [&](const R* v, R* y) { apply_vmass<R>(c, a2, v, y); }, [&](R* v) { project<R>(c, l, v); }, dinv, b, x,
      r, z, p, q, c.par.tol_vmass, c.par.max_inner * 10, 4);
  if (c.rep) c.rep->mass_its += its;
}

// eq. schurWBFBT with the Poisson replacements and the scaled viscosities:
// out = K_{1/sqrt eta_l}^-1 B M_{sqrt eta_l}^-1 A M_{sqrt eta_r}^-1 B^T K_{1/sqrt eta_r}^-1 rp
template <class R>
void schur_wbfbt(Ctx& c, const R* rp, R* out) {
  const int l = c.L();
  LevelData& L = c.at(l);
  const long long N = 3 * L.h.n2, n1 = L.h.n1;
  const double a2l = c.par.a_l * c.par.a_l, a2r = c.par.a_r * c.par.a_r;
  R* y1 = L.ppool<R>().get(Q_WB1, n1, c.s);
  R* y2 = L.ppool<R>().get(Q_WB2, n1, c.s);
  R* t = L.pool<R>().get(W_VM_T, N, c.s);
  R* z = L.pool<R>().get(W_VM_Z2, N, c.s);
  solve_poisson<R>(c, a2r, rp, y1);
  applyBt<R>(c, l, y1, t, false, BCM_OUT);
  solve_vmass<R>(c, a2r, t, z);
  applyA<R>(c, l, z, t, BCM_IN | BCM_OUT);
  if (c.rot) rot_remove<R>(c, t);
  solve_vmass<R>(c, a2l, t, z);
  applyB<R>(c, l, z, y2, false, BCM_IN);
  project_mean<R>(c, y2);
  solve_poisson<R>(c, a2l, y2, out);
}

// S^-1 of the chosen approximation (Sec. 5.2.3) applied to a mean-zero rp
template <class R>
void schur_inv(Ctx& c, const R* rp, R* out) {
  if (c.par.schur == STK_SCHUR_MASS) {
    solve_mass<R>(c, rp, out);   // eq. schurMass
    project_mean<R>(c, out);
    if (c.rep) c.rep->s_solves++;
  } else if (c.par.schur == STK_SCHUR_WBFBT) {
    schur_wbfbt<R>(c, rp, out);   // eq. schurWBFBT
  } else {
    schur_vbfbt<R>(c, rp, out);   // eq. schurV, or the diag(A)-BFBT
  }
}

// Uzawa-type block preconditioners (Sec. 5.2.1), one step from (u, p) = 0:
//   symmetric (eq. SymmetricUzawaStep1):
//     uh = sigma A^-1 ru;  p = -omega S^-1 (rp - Bbar uh);  u = uh + sigma A^-1 (ru - A uh - B^T p)
//   inexact (eq. InexactUzawaStep1):   u = sigma A^-1 ru;  p = -omega S^-1 (rp - Bbar u)
//   adjoint (eq. AdjointInexactUzawaStep1):  p = -omega S^-1 rp;  u = sigma A^-1 (ru - B^T p)
// Bbar = B + C in the pressure update when use_Bbar (Sec. 5.2.1, last remark).
// For the transposed system the roles of B and Bbar swap.
template <class R>
void uzawa(Ctx& c, const R* ru, const R* rp, R* u, R* p, bool transpose) {
  const int l = c.L();
  LevelData& L = c.at(l);
  const long long N = 3 * L.h.n2, n1 = L.h.n1;
  R* uh = L.pool<R>().get(W_U0, N, c.s);
  R* t = L.pool<R>().get(W_U1, N, c.s);
  R* w = L.pool<R>().get(W_U2, N, c.s);
  R* tp = L.ppool<R>().get(Q_U0, n1, c.s);
  R* qp = L.ppool<R>().get(Q_U1, n1, c.s);
  const bool withC = c.has_rho && !transpose && c.par.use_Bbar;
  const bool withCt = c.has_rho && transpose;
  const int variant = c.par.uzawa;
  // p = -omega S^-1 (rp - Bbar v), v = nullptr for v = 0
  auto pressure = [&](const R* v) {
    vcopy<R>(rp, tp, n1, c.s);
    if (v) {
      applyB<R>(c, l, v, qp, withC, BCM_IN);
      vaxpy<R>(R(-1), qp, tp, n1, c.s);
    }
    project_mean<R>(c, tp);
    schur_inv<R>(c, tp, p);
    vscale<R>(R(-c.par.omega), p, n1, c.s);
    project_mean<R>(c, p);
  };
  if (variant == STK_UZAWA_ADJOINT) {
    pressure(nullptr);
    // u = sigma A^-1 (ru - B^T p)
    vcopy<R>(ru, w, N, c.s);
    applyBt<R>(c, l, p, t, withCt, BCM_OUT);
    vaxpy<R>(R(-1), t, w, N, c.s);
    project<R>(c, l, w);
    solve_A<R>(c, w, u);
    if (c.par.sigma != 1.0) vscale<R>(R(c.par.sigma), u, N, c.s);
    return;
  }
  solve_A<R>(c, ru, uh);
  if (c.par.sigma != 1.0) vscale<R>(R(c.par.sigma), uh, N, c.s);
  pressure(uh);
  if (variant == STK_UZAWA_INEXACT) {
    vcopy<R>(uh, u, N, c.s);
    return;
  }
  applyA<R>(c, l, uh, t, BCM_IN | BCM_OUT);
  vcopy<R>(ru, w, N, c.s);
  vaxpy<R>(R(-1), t, w, N, c.s);
  applyBt<R>(c, l, p, t, withCt, BCM_OUT);
  vaxpy<R>(R(-1), t, w, N, c.s);
  project<R>(c, l, w);
  solve_A<R>(c, w, u);
  vaxpby<R>(R(1), uh, R(c.par.sigma), u, N, c.s);
}

// The preconditioner as FGMRES applies it: FP32 (mixed) or FP64 Uzawa step on
// the FP64 residual [v; v + N], result re-projected in FP64
void precondition(Ctx& c, const double* v, double* z, bool transpose) {
  const int l = c.L();
  LevelData& L = c.at(l);
  const long long N = 3 * L.h.n2, n1 = L.h.n1;
  if (c.par.precision == 32) {
    float* vu = L.pool<float>().get(W_F0, N, c.s);
    float* zu = L.pool<float>().get(W_F1, N, c.s);
    float* vp = L.ppool<float>().get(Q_F0, n1, c.s);
    float* zp = L.ppool<float>().get(Q_F1, n1, c.s);
    vconvert<double, float>(v, vu, N, c.s);
    vconvert<double, float>(v + N, vp, n1, c.s);
    uzawa<float>(c, vu, vp, zu, zp, transpose);
    vconvert<float, double>(zu, z, N, c.s);
    vconvert<float, double>(zp, z + N, n1, c.s);
  } else {
    uzawa<double>(c, v, v + N, z, z + N, transpose);
  }
  // keep the Krylov space exactly in range(P): FP32 projections leave
  // normal components of relative size ~1e-7 at free-slip nodes
  project<double>(c, l, z);
  project_mean<double>(c, z + N);
}

// ---- FGMRES (Saad 1993), right preconditioned, FP64 -----------------------------
struct FgmresOut {
  int its = 0;
  double r0 = 0, rfin = 0;
  bool converged = false;
};

// warm: xu, xp enter as the initial guess (projected here); else they start at zero
FgmresOut fgmres(Ctx& c, const double* bu, const double* bp, double* xu, double* xp, bool transpose, bool warm) {
  const int l = c.L();
  LevelData& L = c.at(l);
  const long long N = 3 * L.h.n2, n1 = L.h.n1, Nt = N + n1;
  const int m = c.par.restart;
  // m+1 Krylov vectors V, m preconditioned vectors Z, and the right-hand side
  c.fg.alloc((size_t)(2 * m + 2) * Nt);
  auto V = [&](int j) { return c.fg.p + (size_t)j * Nt; };
  auto Z = [&](int j) { return c.fg.p + (size_t)(m + 1 + j) * Nt; };
  double* b = c.fg.p + (size_t)(2 * m + 1) * Nt;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1);
  auto Hs = [&](int i, int j) -> double& { return H[(size_t)i * m + j]; };
  auto Kapply = [&](const double* x, double* y) {
    applyK<double>(c, x, x + N, y, y + N, transpose, BCM_IN | BCM_OUT);
    if (c.rot) rot_remove<double>(c, y);
    project_mean<double>(c, y + N);
  };
  auto precond = [&](const double* v, double* z) { precondition(c, v, z, transpose); };
  FgmresOut out;
  if (warm) {
    project<double>(c, l, xu);
    project_mean<double>(c, xp);
  } else {
    vfill<double>(xu, 0.0, N, c.s);
    vfill<double>(xp, 0.0, n1, c.s);
  }
  vcopy<double>(bu, b, N, c.s);
  vcopy<double>(bp, b + N, n1, c.s);
  project<double>(c, l, b);
  project_mean<double>(c, b + N);
  const double nb = nrm2<double>(c, b, Nt);
  double beta = nb;
  if (warm) {
    // r0 = b - K x0 (the initial guess, both parts contiguous in Z(0))
    double* tmp = Z(0);
    vcopy<double>(xu, tmp, N, c.s);
    vcopy<double>(xp, tmp + N, n1, c.s);
    Kapply(tmp, V(0));
    vaxpby<double>(1.0, b, -1.0, V(0), Nt, c.s);
    beta = nrm2<double>(c, V(0), Nt);
  } else {
    vcopy<double>(b, V(0), Nt, c.s);
  }
  out.r0 = beta;
  out.rfin = beta;
  if (c.rep) c.rep->initial_residual = beta;
  const double target = std::max(c.par.tol_rel * nb, c.par.tol_abs);
  if (nb == 0.0 || beta <= target) {
    out.converged = true;
    if (nb == 0.0) {
      vfill<double>(xu, 0.0, N, c.s);
      vfill<double>(xp, 0.0, n1, c.s);
    }
    return out;
  }
  int total = 0;
  while (total < c.par.max_outer) {
    vscale<double>(1.0 / beta, V(0), Nt, c.s);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int j_used = 0;
    for (int j = 0; j < m && total < c.par.max_outer; ++j) {
      precond(V(j), Z(j));
      Kapply(Z(j), V(j + 1));
      for (int i = 0; i <= j; ++i) {
        Hs(i, j) = dot<double>(c, V(j + 1), V(i), Nt);
        vaxpy<double>(-Hs(i, j), V(i), V(j + 1), Nt, c.s);
      }
      Hs(j + 1, j) = nrm2<double>(c, V(j + 1), Nt);
      if (Hs(j + 1, j) > 0) vscale<double>(1.0 / Hs(j + 1, j), V(j + 1), Nt, c.s);
      for (int i = 0; i < j; ++i) {
        double t = cs[i] * Hs(i, j) + sn[i] * Hs(i + 1, j);
        Hs(i + 1, j) = -sn[i] * Hs(i, j) + cs[i] * Hs(i + 1, j);
        Hs(i, j) = t;
      }
      double den = std::hypot(Hs(j, j), Hs(j + 1, j));
      cs[j] = Hs(j, j) / den;
      sn[j] = Hs(j + 1, j) / den;
      Hs(j, j) = den;
      Hs(j + 1, j) = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++total;
      j_used = j + 1;
      if (c.rep && c.rep->history_len < 256) c.rep->history[c.rep->history_len++] = std::fabs(g[j + 1]) / nb;
      if (c.verbose) {
        std::fprintf(stderr, "[stk] fgmres it %d rel %.3e  (A its %d, S its %d)\n", total, std::fabs(g[j + 1]) / nb,
                     c.rep ? c.rep->a_cg_its : -1, c.rep ? c.rep->s_cg_its : -1);
        std::fflush(stderr);
      }
      if (std::fabs(g[j + 1]) <= target) break;
    }
    // x += Z y
    std::vector<double> y(j_used);
    for (int i = j_used - 1; i >= 0; --i) {
      double s = g[i];
      for (int k = i + 1; k < j_used; ++k) s -= Hs(i, k) * y[k];
      y[i] = s / Hs(i, i);
    }
    for (int i = 0; i < j_used; ++i) {
      vaxpy<double>(y[i], Z(i), xu, N, c.s);
      vaxpy<double>(y[i], Z(i) + N, xp, n1, c.s);
    }
    // true residual r = b - K x  (into V(0))
    double* tmp = Z(0);
    vcopy<double>(xu, tmp, N, c.s);
    vcopy<double>(xp, tmp + N, n1, c.s);
    Kapply(tmp, V(0));
    vaxpby<double>(1.0, b, -1.0, V(0), Nt, c.s);
    project<double>(c, l, V(0));
    project_mean<double>(c, V(0) + N);
    beta = nrm2<double>(c, V(0), Nt);
    out.rfin = beta;
    out.its = total;
    if (beta <= target) {
      out.converged = true;
      break;
    }
  }
  project<double>(c, l, xu);
  project_mean<double>(c, xp);
  return out;
}

// ---- temperature step (Sec. 3 and Sec. 6, eq. WeakTemp) -----------------------------
// row-major inverse of a 3x3 matrix given row-major
void inv3(const double* A, double* B) {
  const double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                     A[2] * (A[3] * A[7] - A[4] * A[6]);
  REQUIRE(std::fabs(det) > 0.0, "singular 3x3 matrix in the point locator");
  B[0] = (A[4] * A[8] - A[5] * A[7]) / det;
  B[1] = (A[2] * A[7] - A[1] * A[8]) / det;
  B[2] = (A[1] * A[5] - A[2] * A[4]) / det;
  B[3] = (A[5] * A[6] - A[3] * A[8]) / det;
  B[4] = (A[0] * A[8] - A[2] * A[6]) / det;
  B[5] = (A[2] * A[3] - A[0] * A[5]) / det;
  B[6] = (A[3] * A[7] - A[4] * A[6]) / det;
  B[7] = (A[1] * A[6] - A[0] * A[7]) / det;
  B[8] = (A[0] * A[4] - A[1] * A[3]) / det;
}

// Finest-level data of the temperature problem: the Dirichlet node list (both
// spheres, or the cube's boundary) and the point locator of the MMOC.  The
// shell's prism table is built geometrically: each macro-tet's centroid
// direction is classified with the same face / sub-triangle formulas as the
// device locator, its layer is the lowest of its vertices'.
void setup_temp(Ctx& c) {
  if (c.temp.ready) return;
  const Level& h = c.at(c.L()).h;
  std::vector<uint32_t> bn(h.bnode.begin(), h.bnode.end());
  std::vector<uint8_t> bk(h.bkind.begin(), h.bkind.end());
  c.temp.bnode.upload(bn);
  c.temp.bkind.upload(bk);
  c.temp.nb = (int)bn.size();
  LocDev& loc = c.temp.loc;
  loc = LocDev{};
  loc.kind = c.mm.kind;
  for (int t = 0; t < 6; ++t) {
    double A[9];
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) A[3 * r + k] = TYPE_OFF[t][k + 1][r] - TYPE_OFF[t][0][r];
    inv3(A, loc.tinv6[t]);
  }
  const int nm = c.mm.nm();
  std::vector<double> geo = macro_geometry(c.mm);
  std::vector<double> minv((size_t)nm * 9);
  for (int m = 0; m < nm; ++m) inv3(&geo[(size_t)m * 16 + 3], &minv[(size_t)m * 9]);
  c.temp.minv.upload(minv);
  loc.minv = c.temp.minv.p;
  if (c.mm.kind == 1) {
    const int nt = c.desc.n_tan, nr = c.desc.n_rad;
    loc.n_tan = nt;
    loc.n_rad = nr;
    loc.r_in = c.desc.r_in;
    loc.r_out = c.desc.r_out;
    double ico[12][3];
    std::vector<std::array<int, 3>> faces;
    icosahedron(ico, faces);
    for (int f = 0; f < 20; ++f) {
      double A[9];
      for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) A[3 * r + k] = ico[faces[f][k]][r];
      inv3(A, loc.fmat[f]);
    }
    std::vector<int> prism((size_t)20 * 2 * nt * nt * nr * 3, -1);
    for (int m = 0; m < nm; ++m) {
      double cen[3] = {0, 0, 0};
      int lay = 1 << 30;
      for (int v = 0; v < 4; ++v) {
        const int id = c.mm.tets[m][v];
        for (int d = 0; d < 3; ++d) cen[d] += 0.25 * c.mm.V[3 * id + d];
        lay = std::min(lay, c.mm.layer[id]);
      }
      const double r = std::sqrt(cen[0] * cen[0] + cen[1] * cen[1] + cen[2] * cen[2]);
      const double d[3] = {cen[0] / r, cen[1] / r, cen[2] / r};
      int bf = 0;
      double bc[3] = {0, 0, 0}, bmin = -1e300;
      for (int f = 0; f < 20; ++f) {
        const double* M = loc.fmat[f];
        double cc[3];
        for (int k = 0; k < 3; ++k) cc[k] = M[3 * k] * d[0] + M[3 * k + 1] * d[1] + M[3 * k + 2] * d[2];
        const double mn = std::min(cc[0], std::min(cc[1], cc[2]));
        if (mn > bmin) {
          bmin = mn;
          bf = f;
          for (int k = 0; k < 3; ++k) bc[k] = cc[k];
        }
      }
      const double cs = bc[0] + bc[1] + bc[2];
      const double xa = nt * bc[0] / cs, xb = nt * bc[1] / cs;
      const int i = std::min(std::max((int)std::floor(xa), 0), nt - 1);
      const int j = std::min(std::max((int)std::floor(xb), 0), nt - 1 - i);
      const int down = ((xa - i) + (xb - j) > 1.0) && (i + j <= nt - 2);
      const int tri = 2 * (i * nt + j) + down;
      REQUIRE(lay >= 0 && lay < nr, "macro layer out of range");
      int* slot = &prism[(((size_t)bf * 2 * nt * nt + tri) * nr + lay) * 3];
      int s = 0;
      while (s < 3 && slot[s] >= 0) ++s;
      REQUIRE(s < 3, "point locator: more than three macro-tets in one prism");
      slot[s] = m;
    }
    for (int f = 0; f < 20; ++f)
      for (int i = 0; i < nt; ++i)
        for (int j = 0; i + j < nt; ++j)
          for (int down = 0; down < 2; ++down) {
            if (down && i + j > nt - 2) continue;
            for (int k = 0; k < nr; ++k) {
              const int* slot = &prism[(((size_t)f * 2 * nt * nt + 2 * (i * nt + j) + down) * nr + k) * 3];
              REQUIRE(slot[0] >= 0 && slot[1] >= 0 && slot[2] >= 0, "point locator: incomplete prism table");
            }
          }
    c.temp.prism.upload(prism);
    loc.prism = c.temp.prism.p;
  }
  c.temp.ready = true;
}

TempCoef temp_coef(const stk_temp_params& p) {
  TempCoef t{};
  const double t1 = p.tau1, t0 = p.tau0;
  t.s1 = (2.0 * t1 + t0) / (t1 + t0);
  t.s0 = (t1 + t0) / t0;
  t.sm = t1 * t1 / (t0 * (t1 + t0));
  t.tau = t1;
  t.kap = p.k / (p.Pe * p.Cp);
  t.adv = p.adv;
  t.cad = p.Di * p.alpha / p.Cp;
  t.hsrc = p.H / p.Cp;
  t.heat = p.Pe * p.Di / (p.Ra * p.Cp);
  return t;
}

void check_temp_params(const stk_temp_params* p) {
  REQUIRE(p, "null parameters");
  REQUIRE(p->tau1 > 0 && p->tau0 > 0 && std::isfinite(p->tau1) && std::isfinite(p->tau0),
          "time steps tau1, tau0 must be positive");
  REQUIRE(p->Pe != 0 && p->Cp != 0 && p->Ra != 0 && std::isfinite(p->Pe) && std::isfinite(p->Cp) &&
              std::isfinite(p->Ra),
          "Pe, Cp and Ra must be finite and nonzero");
  REQUIRE(p->k >= 0 && std::isfinite(p->k), "k must be finite and >= 0");
  REQUIRE(std::isfinite(p->Di) && std::isfinite(p->alpha) && std::isfinite(p->H) && std::isfinite(p->adv) &&
              std::isfinite(p->T_in) && std::isfinite(p->T_out),
          "non-finite coefficient");
  REQUIRE(p->tol_abs >= 0 && p->tol_cg > 0 && p->tol_cg < 1, "bad tolerances");
  REQUIRE(p->restart >= 1 && p->max_outer >= 1 && p->max_cg >= 1, "restart, max_outer and max_cg must be >= 1");
  REQUIRE(p->stored_S == 0 || p->stored_S == 1, "stored_S must be 0 or 1");
}

// Builds the stored element matrices of S for these coefficients when asked
// for and when their memory (55 doubles per brick slot, about 1.9 slots per
// micro-tet) is free with 2 GiB to spare; returns whether they are in place.
bool temp_build_smat(Ctx& c, const TempCoef& tc, const double* lnrho, bool want) {
  LevelData& L = c.at(c.L());
  const size_t cnt = (size_t)TEMP_SMAT_ENTRIES * temp_smat_slots(L.d);
  if (!want) return false;
  if (c.temp.smat.n != cnt) {
    c.temp.smat.release();
    size_t fr = 0, total = 0;
    HIPCHK(hipMemGetInfo(&fr, &total));
    if (cnt * sizeof(double) + ((size_t)2 << 30) > fr) return false;
    c.temp.smat.alloc(cnt);
  }
  launch_temp_smat(L.d, c.vrule, tc.s1, tc.tau * tc.kap, lnrho, c.temp.smat.p, c.s);
  return true;
}

// temperature work vectors of the finest level (n2 each)
enum { T_US = 0, T_M1, T_M2, T_M3, T_B, T_R, T_D, T_X, T_CR, T_CZ, T_CP, T_CQ, T_TMP, T_NVEC };
double* twork(Ctx& c, int k) {
  const long long n2 = n2of(c, c.L());
  const size_t need = (size_t)(T_NVEC + 2) * n2;   // u* takes 3 n2
  if (c.temp.w.n < need) c.temp.w.alloc(need);
  return c.temp.w.p + (k == T_US ? 0 : (size_t)(k + 2) * n2);
}

void temp_apply(Ctx& c, const TempCoef& tc, int mode, const double* x, const double* u, const double* lnrho,
                double* y) {
  LevelData& L = c.at(c.L());
  launch_temp(L.d, c.vrule, tc, mode, x, u, lnrho, nullptr, nullptr, nullptr, y, c.s);
}
void temp_zero_bc(Ctx& c, double* v) {
  launch_scalar_dirichlet(c.temp.bnode.p, c.temp.bkind.p, c.temp.nb, v, 0, 0.0, 0.0, c.s);
}

// FGMRES (Saad 1993), right preconditioned, for the scalar temperature system
// on the vectors with zero Dirichlet rows; x enters as zero.
template <class Apply, class Prec>
FgmresOut fgmres_scalar(Ctx& c, long long N, Apply apply, Prec prec, const double* b, double* x, double tol_abs,
                        int m, int max_outer) {
  c.temp.fg.alloc((size_t)(2 * m + 1) * N);
  auto V = [&](int j) { return c.temp.fg.p + (size_t)j * N; };
  auto Z = [&](int j) { return c.temp.fg.p + (size_t)(m + 1 + j) * N; };
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1);
  auto Hs = [&](int i, int j) -> double& { return H[(size_t)i * m + j]; };
  FgmresOut out;
  vfill<double>(x, 0.0, N, c.s);
  const double nb = nrm2<double>(c, b, N);
  out.r0 = out.rfin = nb;
  if (nb <= tol_abs || nb == 0.0) {
    out.converged = true;
    return out;
  }
  double beta = nb;
  vcopy<double>(b, V(0), N, c.s);
  int total = 0;
  while (total < max_outer) {
    vscale<double>(1.0 / beta, V(0), N, c.s);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int j_used = 0;
    for (int j = 0; j < m && total < max_outer; ++j) {
      prec(V(j), Z(j));
      apply(Z(j), V(j + 1));
      for (int i = 0; i <= j; ++i) {
        Hs(i, j) = dot<double>(c, V(j + 1), V(i), N);
        vaxpy<double>(-Hs(i, j), V(i), V(j + 1), N, c.s);
      }
      Hs(j + 1, j) = nrm2<double>(c, V(j + 1), N);
      if (Hs(j + 1, j) > 0) vscale<double>(1.0 / Hs(j + 1, j), V(j + 1), N, c.s);
      for (int i = 0; i < j; ++i) {
        double t = cs[i] * Hs(i, j) + sn[i] * Hs(i + 1, j);
        Hs(i + 1, j) = -sn[i] * Hs(i, j) + cs[i] * Hs(i + 1, j);
        Hs(i, j) = t;
      }
      double den = std::hypot(Hs(j, j), Hs(j + 1, j));
      cs[j] = Hs(j, j) / den;
      sn[j] = Hs(j + 1, j) / den;
      Hs(j, j) = den;
      Hs(j + 1, j) = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++total;
      j_used = j + 1;
      if (c.verbose) {
        std::fprintf(stderr, "[stk] temperature fgmres it %d abs %.3e\n", total, std::fabs(g[j + 1]));
        std::fflush(stderr);
      }
      if (std::fabs(g[j + 1]) <= tol_abs) break;
    }
    std::vector<double> yv(j_used);
    for (int i = j_used - 1; i >= 0; --i) {
      double s = g[i];
      for (int k = i + 1; k < j_used; ++k) s -= Hs(i, k) * yv[k];
      yv[i] = s / Hs(i, i);
    }
    for (int i = 0; i < j_used; ++i) vaxpy<double>(yv[i], Z(i), x, N, c.s);
    // true residual b - A x into V(0)
    apply(x, V(0));
    vaxpby<double>(1.0, b, -1.0, V(0), N, c.s);
    beta = nrm2<double>(c, V(0), N);
    out.rfin = beta;
    out.its = total;
    if (beta <= tol_abs) {
      out.converged = true;
      break;
    }
  }
  return out;
}

// T = solution of the Dirichlet problem L T = b, T = T_in / T_out on the
// boundary; T_init (nullable) is the starting guess of the free rows.
void temp_solve(Ctx& c, const stk_temp_params& p, const double* ustar, const double* lnrho, const double* b,
                const double* T_init, double* T, stk_temp_report* rep) {
  setup_temp(c);
  const long long N = n2of(c, c.L());
  const TempCoef tc = temp_coef(p);
  double* dinv = twork(c, T_D);
  double* r = twork(c, T_R);
  double* dx = twork(c, T_X);
  double* tmp = twork(c, T_TMP);
  temp_apply(c, tc, TM_DIAG, nullptr, nullptr, lnrho, tmp);
  vinvert<double>(tmp, dinv, N, c.s);
  const bool stored = temp_build_smat(c, tc, lnrho, p.stored_S == 1);
  LevelData& LF = c.at(c.L());
  if (T_init) vcopy<double>(T_init, T, N, c.s);
  else vfill<double>(T, 0.0, N, c.s);
  launch_scalar_dirichlet(c.temp.bnode.p, c.temp.bkind.p, c.temp.nb, T, 1, p.T_in, p.T_out, c.s);
  temp_apply(c, tc, TM_APPLY, T, ustar, lnrho, tmp);
  vcopy<double>(b, r, N, c.s);
  vaxpy<double>(-1.0, tmp, r, N, c.s);
  temp_zero_bc(c, r);
  int cg_total = 0;
  auto apply = [&](const double* v, double* y) {
    temp_apply(c, tc, TM_APPLY, v, ustar, lnrho, y);
    temp_zero_bc(c, y);
  };
  auto prec = [&](const double* v, double* z) {
    cg_total += dev_pcg<double>(
        c, N, [&](const double* pp, double* q) {
          if (stored) launch_temp_sapply(LF.d, c.temp.smat.p, pp, q, c.s);
          else temp_apply(c, tc, TM_SYM, pp, nullptr, lnrho, q);
          temp_zero_bc(c, q);
        },
        [&](double* w) { temp_zero_bc(c, w); }, dinv, v, z, twork(c, T_CR), twork(c, T_CZ), twork(c, T_CP),
        twork(c, T_CQ), p.tol_cg, p.max_cg, 8);
  };
  FgmresOut fo = fgmres_scalar(c, N, apply, prec, r, dx, p.tol_abs, p.restart, p.max_outer);
  vaxpy<double>(1.0, dx, T, N, c.s);
  HIPCHK(hipStreamSynchronize(c.s));
  if (rep) {
    rep->iterations = fo.its;
    rep->cg_its = cg_total;
    rep->converged = fo.converged ? 1 : 0;
    rep->initial_residual = fo.r0;
    rep->abs_residual = fo.rfin;
    rep->stored_S = stored ? 1 : 0;
  }
  if (!fo.converged) throw StkError(STK_ENOCONV, "temperature FGMRES reached max_outer before tol_abs");
}

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

void temperature_step_internal(Ctx& c, const stk_temp_params* p, const double* T_n, const double* T_nm1,
                               const double* u_n, const double* u_nm1, const double* lnrho, const double* eta,
                               double* T_np1, double* That_n, double* That_nm1, stk_temp_report* rep) {
  check_temp_params(p);
  REQUIRE(T_n && T_nm1 && u_n && u_nm1 && eta && T_np1, "null vector");
  REQUIRE(T_np1 != T_n && T_np1 != T_nm1, "T_np1 must not alias T_n or T_nm1");
  for (const double* o : {That_n, That_nm1})
    REQUIRE(!o || (o != T_n && o != T_nm1 && o != T_np1), "traced outputs must not alias the temperatures");
  REQUIRE(!That_n || That_n != That_nm1, "That_n and That_nm1 must be distinct");
  setup_temp(c);
  if (rep) std::memset(rep, 0, sizeof(*rep));
  const long long n2 = n2of(c, c.L());
  LevelData& L = c.at(c.L());
  double* us = twork(c, T_US);
  double* thn = That_n ? That_n : twork(c, T_M1);
  double* thm = That_nm1 ? That_nm1 : twork(c, T_M2);
  double* mid = twork(c, T_M3);
  double* b = twork(c, T_B);
  auto t0 = std::chrono::steady_clock::now();
  const double q = p->tau1 / p->tau0;
  vcopy<double>(u_n, us, 3 * n2, c.s);
  vaxpby<double>(-q, u_nm1, 1.0 + q, us, 3 * n2, c.s);
  launch_mmoc(L.d, c.temp.loc, T_n, us, u_n, p->tau1, thn, c.s);
  launch_mmoc(L.d, c.temp.loc, T_nm1, u_n, u_nm1, p->tau0, mid, c.s);
  launch_mmoc(L.d, c.temp.loc, mid, us, u_n, p->tau1, thm, c.s);
  HIPCHK(hipStreamSynchronize(c.s));
  const double ms_mmoc = ms_since(t0);
  t0 = std::chrono::steady_clock::now();
  launch_temp(L.d, c.vrule, temp_coef(*p), TM_RHS, nullptr, us, lnrho, eta, thn, thm, b, c.s);
  HIPCHK(hipStreamSynchronize(c.s));
  const double ms_rhs = ms_since(t0);
  t0 = std::chrono::steady_clock::now();
  stk_temp_report local{};
  try {
    temp_solve(c, *p, us, lnrho, b, T_n, T_np1, &local);
  } catch (...) {
    local.ms_mmoc = ms_mmoc;
    local.ms_rhs = ms_rhs;
    local.ms_solve = ms_since(t0);
    if (rep) *rep = local;
    throw;
  }
  local.ms_mmoc = ms_mmoc;
  local.ms_rhs = ms_rhs;
  local.ms_solve = ms_since(t0);
  if (rep) *rep = local;
}

// ---- setup --------------------------------------------------------------------------
// Coarsest level: the element node table, the node-to-element incidence slots and
// the per-node boundary data of the element-matrix CG.  The element order is
// that of the level's element list (macro-major), as in the element kernels.
void setup_coarse(Ctx& c, LevelData& L, const std::vector<int>& ea) {
  const Level& h = L.h;
  const int n = h.n, m2 = 2 * n, nm = c.mm.nm();
  const long long ne = (long long)ea.size() * nm;
  const long long nn = h.n2;
  REQUIRE(nn <= 256LL * DOT_BLOCKS && ne * 900 * 8 <= (4LL << 30),
          "min_level too fine: the coarsest level must have at most 262144 P2 nodes and 596523 micro-tets");
  std::vector<uint32_t> en((size_t)ne * 10);
  for (int mac = 0; mac < nm; ++mac)
    for (size_t k = 0; k < ea.size(); ++k) {
      const int pk = ea[k];
      const int t = pk & 7, px = (pk >> 3) & 1023, py = (pk >> 13) & 1023, pz = pk >> 23;
      int P[10][3];
      for (int v = 0; v < 4; ++v)
        for (int d = 0; d < 3; ++d) P[v][d] = 2 * ((d == 0 ? px : d == 1 ? py : pz) + TYPE_OFF[t][v][d]);
      for (int e = 0; e < 6; ++e)
        for (int d = 0; d < 3; ++d) P[4 + e][d] = (P[EDGE_V[e][0]][d] + P[EDGE_V[e][1]][d]) / 2;
      uint32_t* out = en.data() + ((size_t)mac * ea.size() + k) * 10;
      for (int a = 0; a < 10; ++a)
        out[a] = h.l2g2[(size_t)mac * h.nloc2 + lattice_loc(P[a][0], P[a][1], P[a][2], m2)];
    }
  std::vector<int> ptr(nn + 1, 0), pos((size_t)ne * 10);
  for (size_t i = 0; i < en.size(); ++i) ptr[en[i] + 1]++;
  for (long long i = 0; i < nn; ++i) ptr[i + 1] += ptr[i];
  {
    std::vector<int> fill(ptr.begin(), ptr.end() - 1);
    for (size_t i = 0; i < en.size(); ++i) pos[i] = fill[en[i]]++;
  }
  std::vector<uint8_t> act(nn, ACT_NONE);
  std::vector<double> nrm(3 * nn, 0.0);
  for (size_t i = 0; i < h.bnode.size(); ++i) {
    const int bc = h.bkind[i] == 1 ? c.desc.bc_inner : c.desc.bc_outer;
    const uint32_t g = h.bnode[i];
    if (bc == STK_BC_DIRICHLET) {
      act[g] = ACT_DIR;
    } else if (bc == STK_BC_FREESLIP) {
      act[g] = ACT_FS;
      for (int k = 0; k < 3; ++k) nrm[3 * (size_t)g + k] = h.bnormal[3 * i + k];
    }
  }
  L.c_enode.upload(en);
  L.c_iptr.upload(ptr);
  L.c_pos.upload(pos);
  L.c_act.upload(act);
  L.c_nrm.upload(nrm);
  L.c_emat.alloc((size_t)ne * 900);
  L.c_ematf.alloc((size_t)ne * 900);
  L.cd = CoarseDev{(int)ne, (int)nn, L.c_enode.p, L.c_emat.p, L.c_ematf.p, L.c_iptr.p, L.c_pos.p, L.c_act.p,
                   L.c_nrm.p, nullptr};
  L.ccg = true;
}

void upload_level(Ctx& c, int l) {
  LevelData& L = c.at(l);
  const Level& h = L.h;
  L.l2g2.upload(h.l2g2);
  L.l2g1.upload(h.l2g1);
  L.tinv.upload(h.tinv);
  std::vector<float> tf(h.tinv.begin(), h.tinv.end());
  L.tinvf.upload(tf);
  L.tiles.upload(h.tiles);
  LevelDev& d = L.d;
  d.n = h.n;
  d.nloc2 = (int)h.nloc2;
  d.nloc1 = (int)h.nloc1;
  d.nmacro = c.mm.nm();
  d.ntiles = (int)h.tiles.size() / 3;
  d.blend = c.mm.kind == 1;
  d.n2 = h.n2;
  d.n1 = h.n1;
  d.l2g2 = L.l2g2.p;
  d.l2g1 = L.l2g1.p;
  d.geo = c.geo.p;
  d.geof = c.geof.p;
  d.tinv = L.tinv.p;
  d.tinvf = L.tinvf.p;
  d.bact = c.bact.p;
  d.own = c.own.p;
  d.tiles = L.tiles.p;
  // plane-sweep tables: as many strips as needed to keep the fused FP64
  // kernel's LDS ring within 64 KiB
  for (int ns = 1;; ns *= 2) {
    L.sw = build_sweep(h.n, ns);
    if (sweep_lds_bytes(F_A | F_BT | F_B | F_C, L.sw.cap2, L.sw.cap1, 8) <= 65536 || ns >= h.n) break;
  }
  {
    std::vector<int> ea;
    for (int t = 0; t < 6; ++t) {
      const int lim = t == 0 ? h.n - 1 : (t == 5 ? h.n - 3 : h.n - 2);
      for (int pz = 0; pz < h.n; ++pz)
        for (int py = 0; py < h.n; ++py)
          for (int px = 0; px + py + pz <= lim; ++px) ea.push_back(t | (px << 3) | (py << 13) | (pz << 23));
    }
    L.eall.upload(ea);
    d.eall = L.eall.p;
    d.elemwise = h.n <= 2;
    if (l == c.lmin()) setup_coarse(c, L, ea);
  }
  L.sw_strip.upload(L.sw.strip);
  L.sw_plist2.upload(L.sw.plist2);
  L.sw_poff2.upload(L.sw.poff2);
  L.sw_plist1.upload(L.sw.plist1);
  L.sw_poff1.upload(L.sw.poff1);
  L.sw_elist.upload(L.sw.elist);
  L.sw_eoff.upload(L.sw.eoff);
  L.sw_etab.upload(L.sw.etab);
  d.sw.nstrips = L.sw.nstrips;
  d.sw.cap2 = L.sw.cap2;
  d.sw.cap1 = L.sw.cap1;
  d.sw.nsh2 = L.sw.nsh2;
  d.sw.nsh1 = L.sw.nsh1;
  d.sw.strip = L.sw_strip.p;
  d.sw.plist2 = (const int2*)L.sw_plist2.p;
  d.sw.poff2 = L.sw_poff2.p;
  d.sw.plist1 = (const int2*)L.sw_plist1.p;
  d.sw.poff1 = L.sw_poff1.p;
  d.sw.elist = L.sw_elist.p;
  d.sw.eoff = L.sw_eoff.p;
  d.sw.etab = (const int4*)L.sw_etab.p;
  {
    // global node of every plane-list entry of every macro, in plane-list order
    const int nm = c.mm.nm();
    const size_t ne2 = L.sw.plist2.size() / 2, ne1 = L.sw.plist1.size() / 2;
    std::vector<uint32_t> t2(ne2 * nm), t1(ne1 * nm);
    std::vector<int64_t> loc2(ne2), loc1(ne1);
    for (size_t e = 0; e < ne2; ++e) {
      const int pk = L.sw.plist2[2 * e];
      loc2[e] = lattice_loc(pk & 1023, (pk >> 10) & 1023, pk >> 20, 2 * h.n);
    }
    for (size_t e = 0; e < ne1; ++e) {
      const int pk = L.sw.plist1[2 * e];
      loc1[e] = lattice_loc(pk & 1023, (pk >> 10) & 1023, pk >> 20, h.n);
    }
    for (int mc = 0; mc < nm; ++mc) {
      const uint32_t* a2 = h.l2g2.data() + (size_t)mc * h.nloc2;
      const uint32_t* a1 = h.l2g1.data() + (size_t)mc * h.nloc1;
      for (size_t e = 0; e < ne2; ++e) t2[(size_t)mc * ne2 + e] = a2[loc2[e]];
      for (size_t e = 0; e < ne1; ++e) t1[(size_t)mc * ne1 + e] = a1[loc1[e]];
    }
    L.sw_g2tab.upload(t2);
    L.sw_g1tab.upload(t1);
    d.sw.ne2 = (int)ne2;
    d.sw.ne1 = (int)ne1;
    d.sw.g2tab = L.sw_g2tab.p;
    d.sw.g1tab = L.sw_g1tab.p;
  }
  {
    std::vector<uint32_t> node;
    std::vector<int> ptr, slot;
    build_gather(c.mm, h, L.sw, 2, node, ptr, slot);
    L.g2node.upload(node);
    L.g2ptr.upload(ptr);
    L.g2slot.upload(slot);
    d.g2 = GatherDev{(int)node.size(), L.g2node.p, L.g2ptr.p, L.g2slot.p};
    build_gather(c.mm, h, L.sw, 1, node, ptr, slot);
    L.g1node.upload(node);
    L.g1ptr.upload(ptr);
    L.g1slot.upload(slot);
    d.g1 = GatherDev{(int)node.size(), L.g1node.p, L.g1ptr.p, L.g1slot.p};
  }
  // grid-transfer table (this level as the coarse one)
  {
    TransferTable tt = build_transfer_table(h);
    L.xt_tab.upload(tt.tab);
    L.xt_off.upload(tt.off);
    d.xtab = (const int4*)L.xt_tab.p;
    d.xoff = L.xt_off.p;
  }
  // P1 mass stencil (used where a macro's P1 lattice fits the LDS staging)
  {
    P1Stencil ps = build_p1_stencil(h.n);
    L.ms_nb.upload(ps.nb);
    L.ms_dst.upload(ps.dst);
    L.ms_incptr.upload(ps.inc_ptr);
    L.ms_inc.upload(ps.inc);
    std::vector<uint32_t> node;
    std::vector<int> ptr, slot;
    build_gather(c.mm, h, ps.slots, 1, node, ptr, slot);
    L.ms_gnode.upload(node);
    L.ms_gptr.upload(ptr);
    L.ms_gslot.upload(slot);
    StencilDev& m = d.ms;
    m.on = mass_stencil_lds_bytes((int)h.nloc1, 8) <= 65536;
    m.nsh = ps.nsh;
    m.nb = L.ms_nb.p;
    m.dst = L.ms_dst.p;
    m.inc_ptr = L.ms_incptr.p;
    m.inc = (const int2*)L.ms_inc.p;
    m.c64 = nullptr;
    m.c32 = nullptr;
    m.g = GatherDev{(int)node.size(), L.ms_gnode.p, L.ms_gptr.p, L.ms_gslot.p};
  }
  // boundary lists
  std::vector<uint32_t> dir, fs;
  std::vector<double> nrm;
  for (size_t i = 0; i < h.bnode.size(); ++i) {
    const int kind = h.bkind[i];
    const int bc = kind == 1 ? c.desc.bc_inner : c.desc.bc_outer;
    if (bc == STK_BC_DIRICHLET) {
      dir.push_back(h.bnode[i]);
    } else if (bc == STK_BC_FREESLIP) {
      fs.push_back(h.bnode[i]);
      for (int k = 0; k < 3; ++k) nrm.push_back(h.bnormal[3 * i + k]);
    }
  }
  L.dir.upload(dir);
  L.fs.upload(fs);
  L.nrm.upload(nrm);
  std::vector<float> nf(nrm.begin(), nrm.end());
  L.nrmf.upload(nf);
  L.bc.ndir = (int)dir.size();
  L.bc.nfs = (int)fs.size();
  L.bc.dir = L.dir.p;
  L.bc.fs = L.fs.p;
  L.bc.nrm = L.nrm.p;
  L.bc.nrmf = L.nrmf.p;
}

void check_params(const stk_solver_params* p) {
  REQUIRE(p, "null solver parameters");
  REQUIRE(p->precision == 32 || p->precision == 64, "precision must be 32 or 64");
  REQUIRE(p->restart >= 1 && p->restart <= 200, "restart out of range");
  REQUIRE(p->m_A >= 1 && p->deg_A >= 1 && p->m_V >= 1 && p->deg_V >= 1, "smoother steps/degree must be >= 1");
  REQUIRE(p->cheb_lo > 0 && p->cheb_hi > p->cheb_lo, "bad Chebyshev interval factors");
  REQUIRE(p->max_inner >= 1 && p->max_outer >= 1 && p->power_its >= 1, "iteration caps must be >= 1");
  REQUIRE(p->uzawa >= STK_UZAWA_SYMMETRIC && p->uzawa <= STK_UZAWA_ADJOINT, "unknown Uzawa variant");
  REQUIRE(p->schur >= STK_SCHUR_VBFBT && p->schur <= STK_SCHUR_WBFBT, "unknown Schur approximation");
  if (p->schur == STK_SCHUR_WBFBT)
    REQUIRE(p->a_l > 0 && p->a_r > 0 && p->tol_wbfbt > 0 && p->tol_vmass > 0,
            "w-BFBT needs a_l, a_r, tol_wbfbt, tol_vmass > 0");
  REQUIRE(p->initial_guess == 0 || p->initial_guess == 1, "initial_guess must be 0 or 1");
}

// Gauss-Jacobi rule with k points for the weight (1 - x)^alpha on [-1, 1]
// (Golub-Welsch: the nodes are the eigenvalues of the Jacobi matrix of the
// three-term recurrence, the weights mu0 times the squared first eigenvector
// components), eigenvalues by cyclic Jacobi rotations.
void gauss_jacobi(int k, double alpha, double* x, double* w) {
  const double beta = 0.0, ab = alpha + beta;
  std::vector<double> J((size_t)k * k, 0.0), V((size_t)k * k, 0.0);
  for (int i = 0; i < k; ++i) {
    const double d = 2.0 * i + ab;
    J[(size_t)i * k + i] = (i == 0) ? (beta - alpha) / (ab + 2.0) : (beta * beta - alpha * alpha) / (d * (d + 2.0));
    if (i > 0) {
      const double b = std::sqrt(4.0 * i * (i + alpha) * (i + beta) * (i + ab) / (d * d * (d + 1.0) * (d - 1.0)));
      J[(size_t)i * k + i - 1] = J[(size_t)(i - 1) * k + i] = b;
    }
    V[(size_t)i * k + i] = 1.0;
  }
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < k; ++p)
      for (int q = p + 1; q < k; ++q) off += J[(size_t)p * k + q] * J[(size_t)p * k + q];
    if (off < 1e-32) break;
    for (int p = 0; p < k; ++p)
      for (int q = p + 1; q < k; ++q) {
        const double apq = J[(size_t)p * k + q];
        if (apq == 0.0) continue;
        const double theta = (J[(size_t)q * k + q] - J[(size_t)p * k + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int r = 0; r < k; ++r) {   // J <- J G (columns p, q)
          const double jp = J[(size_t)r * k + p], jq = J[(size_t)r * k + q];
          J[(size_t)r * k + p] = cs * jp - sn * jq;
          J[(size_t)r * k + q] = sn * jp + cs * jq;
        }
        for (int r = 0; r < k; ++r) {   // J <- G^T J (rows p, q)
          const double jp = J[(size_t)p * k + r], jq = J[(size_t)q * k + r];
          J[(size_t)p * k + r] = cs * jp - sn * jq;
          J[(size_t)q * k + r] = sn * jp + cs * jq;
        }
        for (int r = 0; r < k; ++r) {   // V <- V G
          const double vp = V[(size_t)r * k + p], vq = V[(size_t)r * k + q];
          V[(size_t)r * k + p] = cs * vp - sn * vq;
          V[(size_t)r * k + q] = sn * vp + cs * vq;
        }
      }
  }
  const double mu0 = std::pow(2.0, ab + 1.0) * std::tgamma(alpha + 1.0) * std::tgamma(beta + 1.0) / std::tgamma(ab + 2.0);
  for (int i = 0; i < k; ++i) {
    x[i] = J[(size_t)i * k + i];
    w[i] = mu0 * V[i] * V[i];   // first row of the eigenvector matrix
  }
}

// The 27-point conical-product rule on the reference tetrahedron (3 Gauss-
// Jacobi points with weights (1 - u)^2, (1 - u), 1 per collapsed direction;
// exact to degree 5), as barycentric points; checked against the monomial
// integrals a! b! c! / (a + b + c + 3)! up to degree 5.
VmassRule make_vmass_rule() {
  double u[3][3], wu[3][3];
  const double alphas[3] = {2.0, 1.0, 0.0};
  for (int d = 0; d < 3; ++d) {
    double x[3], w[3];
    gauss_jacobi(3, alphas[d], x, w);
    for (int i = 0; i < 3; ++i) {
      u[d][i] = 0.5 * (1.0 + x[i]);
      wu[d][i] = w[i] / std::pow(2.0, alphas[d] + 1.0);
    }
  }
  VmassRule r{};
  int q = 0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k, ++q) {
        const double x1 = u[0][i], x2 = (1.0 - u[0][i]) * u[1][j], x3 = (1.0 - u[0][i]) * (1.0 - u[1][j]) * u[2][k];
        r.lam[q][0] = 1.0 - x1 - x2 - x3;
        r.lam[q][1] = x1;
        r.lam[q][2] = x2;
        r.lam[q][3] = x3;
        r.w[q] = wu[0][i] * wu[1][j] * wu[2][k];
      }
  auto fact = [](int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
  };
  for (int a = 0; a <= 5; ++a)
    for (int b = 0; a + b <= 5; ++b)
      for (int c = 0; a + b + c <= 5; ++c) {
        double sum = 0.0;
        for (int p = 0; p < VMASS_NQ; ++p)
          sum += r.w[p] * std::pow(r.lam[p][1], a) * std::pow(r.lam[p][2], b) * std::pow(r.lam[p][3], c);
        const double exact = fact(a) * fact(b) * fact(c) / fact(a + b + c + 3);
        REQUIRE(std::fabs(sum - exact) <= 1e-14, "vector-mass quadrature rule failed its exactness check");
      }
  return r;
}

// power iteration for lambda_max(D^-1 A) with projections, FP64
double power_lambda(Ctx& c, int l, int its) {
  LevelData& L = c.at(l);
  const long long N = 3 * L.h.n2;
  Pool<double>& P = L.pool<double>();
  double* x = P.get(W_CG_R, N, c.s);
  double* t = P.get(W_CG_Z, N, c.s);
  std::vector<double> hx(N);
  uint64_t st = 0x9E3779B97F4A7C15ull ^ (uint64_t)l;
  for (long long i = 0; i < N; ++i) {   // splitmix64, uniform in [-1, 1)
    st += 0x9E3779B97F4A7C15ull;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    hx[i] = (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
  }
  HIPCHK(hipMemcpyAsync(x, hx.data(), N * sizeof(double), hipMemcpyHostToDevice, c.s));
  project<double>(c, l, x);
  double nx = nrm2<double>(c, x, N);
  vscale<double>(1.0 / nx, x, N, c.s);
  double lam = 0;
  for (int it = 0; it < its; ++it) {
    applyA<double>(c, l, x, t, BCM_IN | BCM_OUT);
    vmul<double>(L.dinv.p, t, x, N, c.s);
    project<double>(c, l, x);
    lam = nrm2<double>(c, x, N);
    vscale<double>(1.0 / lam, x, N, c.s);
  }
  return lam;
}

void set_fields_internal(Ctx& c, const double* eta, const double* lnrho, const stk_solver_params* par) {
  check_params(par);
  c.par = *par;
  ++c.field_gen;   // the weighted-BFBT operators of earlier fields are stale
  const int Lf = c.L();
  LevelData& F = c.at(Lf);
  const long long n1 = F.h.n1;
  // validate eta > 0, finite
  {
    std::vector<double> h(n1);
    HIPCHK(hipMemcpyAsync(h.data(), eta, n1 * sizeof(double), hipMemcpyDeviceToHost, c.s));
    HIPCHK(hipStreamSynchronize(c.s));
    for (long long i = 0; i < n1; ++i)
      REQUIRE(std::isfinite(h[i]) && h[i] > 0.0, "viscosity must be positive and finite");
  }
  for (int l = c.lmin(); l <= Lf; ++l) {
    LevelData& L = c.at(l);
    L.eta.alloc(L.h.n1);
    L.etaf.alloc(L.h.n1);
  }
  if (eta != F.eta.p) vcopy<double>(eta, F.eta.p, n1, c.s);
  for (int l = Lf; l > c.lmin(); --l) launch_inject<double>(c.at(l - 1).d, c.at(l).d, c.at(l).eta.p, c.at(l - 1).eta.p, c.s);
  c.has_rho = lnrho != nullptr;
  if (lnrho) {
    c.lnrho.alloc(n1);
    c.lnrhof.alloc(n1);
    vcopy<double>(lnrho, c.lnrho.p, n1, c.s);
    vconvert<double, float>(c.lnrho.p, c.lnrhof.p, n1, c.s);
  }
  for (int l = c.lmin(); l <= Lf; ++l) {
    LevelData& L = c.at(l);
    const long long N = 3 * L.h.n2;
    vconvert<double, float>(L.eta.p, L.etaf.p, L.h.n1, c.s);
    L.dinv.alloc(N);
    L.dinvf.alloc(N);
    vfill<double>(L.dinv.p, 0.0, N, c.s);
    if (L.d.qpv) launch_elem_diag(L.d, L.eta.p, L.dinv.p, c.s);
    else launch_diag<double>(L.d, L.eta.p, L.dinv.p, c.s);
    vinvert<double>(L.dinv.p, L.dinv.p, N, c.s);
    vconvert<double, float>(L.dinv.p, L.dinvf.p, N, c.s);
  }
  {
    LevelData& C = c.at(c.lmin());
    if (C.ccg) {
      C.cd.dinv = C.dinv.p;
      launch_elem_matrix(C.d, C.eta.p, C.c_emat.p, C.c_ematf.p, c.s);
    }
  }
  for (int l = c.lmin() + 1; l <= Lf; ++l) {
    LevelData& L = c.at(l);
    if (!L.bounds_set) {
      const double lam = power_lambda(c, l, par->power_its);
      L.lo = par->cheb_lo * lam;
      L.hi = par->cheb_hi * lam;
    }
  }
  // P1 mass stencils
  for (int l = c.lmin(); l <= Lf; ++l) {
    LevelData& L = c.at(l);
    if (!L.d.ms.on) continue;
    const size_t nc = (size_t)L.d.nmacro * NSTORE1 * (L.h.nloc1 + 1);
    L.ms_c64.alloc(nc);
    L.ms_c32.alloc(nc);
    L.d.ms.c64 = L.ms_c64.p;
    L.d.ms.c32 = L.ms_c32.p;
    launch_mass_stencil_build(L.d, L.eta.p, L.ms_c64.p, L.ms_c32.p, c.s);
  }
  // inverse diagonal of M_{1/eta} (Jacobi preconditioner of its CG)
  {
    double* md = F.ppool<double>().get(Q_MD, n1, c.s);
    vfill<double>(md, 0.0, n1, c.s);
    launch_mass_diag(F.d, F.eta.p, md, c.s);
    vinvert<double>(md, md, n1, c.s);
    float* mdf = F.ppool<float>().get(Q_MD, n1, c.s);
    vconvert<double, float>(md, mdf, n1, c.s);
  }
  HIPCHK(hipStreamSynchronize(c.s));
  HIPCHK(hipGetLastError());
  c.ready = true;
}

// Levels min_level .. l_eta take the quadrature-point viscosity and the
// element-parallel kernel; the others the P1 viscosity and the plane sweep on
// levels with n > 2.
void configure_viscosity_levels(Ctx& c, int l_eta) {
  for (int l = c.lmin(); l <= c.L(); ++l) {
    LevelDev& d = c.at(l).d;
    d.qpv = l <= l_eta ? 1 : 0;
    d.elemwise = (c.at(l).h.n <= 2 || l <= l_eta) ? 1 : 0;
  }
}

void set_temperature_viscosity_internal(Ctx& c, const double* T2, const double* lnrho, const double* base, int nbase,
                                        double EA, double VA, int l_eta, const stk_solver_params* par) {
  REQUIRE(c.desc.kind == STK_MESH_SHELL, "quadrature-point viscosity needs the blended shell");
  REQUIRE(l_eta < c.L(), "l_eta must be below the finest level");
  REQUIRE(nbase >= 2, "eta_base needs at least two samples");
  for (int i = 0; i < nbase; ++i) REQUIRE(std::isfinite(base[i]) && base[i] > 0.0, "eta_base must be positive");
  REQUIRE(std::isfinite(EA) && std::isfinite(VA), "E_A and V_A must be finite");
  check_params(par);
  const int Lf = c.L();
  LevelData& F = c.at(Lf);
  const long long n2 = F.h.n2;
  {
    std::vector<double> h(n2);
    HIPCHK(hipMemcpyAsync(h.data(), T2, n2 * sizeof(double), hipMemcpyDeviceToHost, c.s));
    HIPCHK(hipStreamSynchronize(c.s));
    for (long long i = 0; i < n2; ++i) REQUIRE(std::isfinite(h[i]), "temperature must be finite");
  }
  c.vbase.upload(std::vector<double>(base, base + nbase));
  const ViscDev vm{c.vbase.p, nbase, EA, VA, c.desc.r_in, c.desc.r_out};
  for (int l = c.lmin(); l <= Lf; ++l) {
    LevelData& L = c.at(l);
    L.T2.alloc(L.h.n2);
    L.T2f.alloc(L.h.n2);
    L.d.T2 = L.T2.p;
    L.d.T2f = L.T2f.p;
    L.d.vm = vm;
  }
  vcopy<double>(T2, F.T2.p, n2, c.s);
  for (int l = Lf; l > c.lmin(); --l) launch_inject_p2<double>(c.at(l - 1).d, c.at(l).d, c.at(l).T2.p, c.at(l - 1).T2.p, c.s);
  for (int l = c.lmin(); l <= Lf; ++l) vconvert<double, float>(c.at(l).T2.p, c.at(l).T2f.p, c.at(l).h.n2, c.s);
  configure_viscosity_levels(c, l_eta);
  F.eta.alloc(F.h.n1);
  launch_eta_vertices(F.d, F.eta.p, c.s);
  set_fields_internal(c, F.eta.p, lnrho, par);
}

// Node counts of the finest level in closed form (Sec. 4.1: N = n_tan 2^L
// points per icosahedron edge and M = n_rad 2^L radial intervals give
// (10 (2N)^2 + 2)(2M + 1) P2 and (10 N^2 + 2)(M + 1) P1 nodes on the shell;
// the cube has (2^{L+1} + 1)^3 and (2^L + 1)^3), computed in long double so
// that no descriptor overflows them.
void closed_form_counts(const stk_mesh_desc& d, long double& n2, long double& n1) {
  const long double s = std::ldexp(1.0L, d.level);
  if (d.kind == STK_MESH_CUBE) {
    n2 = std::pow(2.0L * s + 1.0L, 3);
    n1 = std::pow(s + 1.0L, 3);
  } else {
    const long double N = (long double)d.n_tan * s, M = (long double)d.n_rad * s;
    n2 = (10.0L * 4.0L * N * N + 2.0L) * (2.0L * M + 1.0L);
    n1 = (10.0L * N * N + 2.0L) * (M + 1.0L);
  }
}

void need_ready(Ctx* c) {
  REQUIRE(c, "null context");
  if (!c->ready) throw StkError(STK_ENOTREADY, "stk_set_fields has not been called");
}
void check_level(Ctx* c, int level) {
  REQUIRE(c, "null context");
  REQUIRE(level >= c->lmin() && level <= c->L(), "level outside [min_level, level]");
}

}  // namespace

// =====================================================================================
extern "C" {

const char* stk_last_error(void) { return g_err.c_str(); }

void stk_default_params(stk_solver_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->tol_rel = 1e-8;
  p->tol_abs = 0.0;
  p->restart = 20;
  p->max_outer = 200;
  p->precision = 64;
  p->sigma = 1.0;
  p->omega = 0.3;
  p->tol_A = 1e-2;
  p->tol_vbfbt = 1e-1;
  p->tol_invmass = 1e-10;
  p->tol_coarse = 1e-2;
  p->m_A = 3;
  p->deg_A = 2;
  p->m_V = 1;
  p->deg_V = 1;
  p->max_inner = 100;
  p->use_Bbar = 1;
  p->power_its = 15;
  p->cheb_lo = 0.12;
  p->cheb_hi = 1.2;
  p->a_l = 1.0;
  p->a_r = 1.0;
  p->tol_wbfbt = 1e-10;
  p->tol_vmass = 1e-4;
  p->initial_guess = 0;
}

int stk_create(const stk_mesh_desc* desc, void* hip_stream, stk_ctx** out) {
  return guard([&] {
    REQUIRE(desc && out, "null argument");
    REQUIRE(desc->kind == STK_MESH_CUBE || desc->kind == STK_MESH_SHELL, "unknown mesh kind");
    REQUIRE(desc->level >= 0 && desc->level <= 7, "level must be in [0, 7]");
    REQUIRE(desc->min_level >= 0 && desc->min_level <= desc->level, "min_level must be in [0, level]");
    REQUIRE(desc->bc_inner == STK_BC_DIRICHLET || desc->bc_inner == STK_BC_FREESLIP, "bad bc_inner");
    if (desc->kind == STK_MESH_CUBE) {
      REQUIRE(desc->bc_inner == STK_BC_DIRICHLET, "the cube supports Dirichlet boundaries only");
    } else {
      REQUIRE(desc->bc_outer == STK_BC_DIRICHLET || desc->bc_outer == STK_BC_FREESLIP, "bad bc_outer");
      REQUIRE(desc->n_tan >= 1 && desc->n_rad >= 1, "n_tan and n_rad must be >= 1");
      REQUIRE(desc->r_in > 0 && desc->r_out > desc->r_in, "need 0 < r_in < r_out");
    }
    {
      // the kernels index nodes with signed 32-bit integers (shared nodes of
      // a macro are encoded as negative slot numbers), so both node counts
      // must stay below 2^31
      long double n2, n1;
      closed_form_counts(*desc, n2, n1);
      REQUIRE(n2 < 2147483648.0L && n1 < 2147483648.0L,
              "mesh too large: the P2 and P1 node counts must be below 2^31");
    }
    std::unique_ptr<stk_ctx> c(new stk_ctx());
    c->desc = *desc;
    c->s = (hipStream_t)hip_stream;
    HIPCHK(hipGetDevice(&c->device));
    c->vrule = make_vmass_rule();
    HIPCHK(noalloc_scratch_init(c->device));   // address of this GPU's fixed scratch array
    c->mm = desc->kind == STK_MESH_CUBE ? make_cube() : make_shell(desc->n_tan, desc->n_rad, desc->r_in, desc->r_out);
    c->top = build_topology(c->mm);
    std::vector<double> geo = macro_geometry(c->mm);
    c->geo.upload(geo);
    std::vector<float> gf(geo.begin(), geo.end());
    c->geof.upload(gf);
    // BC action per macro and node class
    std::vector<uint8_t> act(c->top.bkind.size());
    for (size_t i = 0; i < act.size(); ++i) {
      const int k = c->top.bkind[i];
      act[i] = k == 0 ? ACT_NONE : (uint8_t)(k == 1 ? desc->bc_inner : desc->bc_outer);
    }
    c->bact.upload(act);
    c->own.upload(c->top.own);
    c->lv.resize(desc->level + 1);
    for (int l = desc->min_level; l <= desc->level; ++l) {
      c->lv[l].reset(new LevelData());
      c->lv[l]->h = build_level(c->mm, c->top, l);
      upload_level(*c, l);
    }
    if (desc->kind == STK_MESH_SHELL && desc->bc_inner == STK_BC_FREESLIP && desc->bc_outer == STK_BC_FREESLIP) {
      // the rigid rotations e_k x X: node positions of the finest level and
      // the inverse of their Gram matrix G = sum_i (|X_i|^2 I - X_i X_i^T)
      const Level& h = c->lv[desc->level]->h;
      std::vector<double> X((size_t)3 * h.n2);
      level_coords(c->mm, c->top, h, 2, X.data(), nullptr);
      double G[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
      for (long long i = 0; i < h.n2; ++i) {
        const double* x = &X[3 * i];
        const double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) G[3 * a + b] += (a == b ? r2 : 0.0) - x[a] * x[b];
      }
      const double det = G[0] * (G[4] * G[8] - G[5] * G[7]) - G[1] * (G[3] * G[8] - G[5] * G[6]) +
                         G[2] * (G[3] * G[7] - G[4] * G[6]);
      REQUIRE(det > 0, "degenerate node set for the rotation constraint");
      double* gi = c->rotd.gi;
      gi[0] = (G[4] * G[8] - G[5] * G[7]) / det;
      gi[1] = (G[2] * G[7] - G[1] * G[8]) / det;
      gi[2] = (G[1] * G[5] - G[2] * G[4]) / det;
      gi[3] = (G[5] * G[6] - G[3] * G[8]) / det;
      gi[4] = (G[0] * G[8] - G[2] * G[6]) / det;
      gi[5] = (G[2] * G[3] - G[0] * G[5]) / det;
      gi[6] = (G[3] * G[7] - G[4] * G[6]) / det;
      gi[7] = (G[1] * G[6] - G[0] * G[7]) / det;
      gi[8] = (G[0] * G[4] - G[1] * G[3]) / det;
      c->rotX.upload(X);
      c->rotbuf.alloc(3 * DOT_BLOCKS);
      c->rotd.X = c->rotX.p;
      c->rot = true;
    }
    c->dotbuf.alloc(2 * DOT_BLOCKS + 8);
    c->meanbuf.alloc(DOT_BLOCKS);
    c->cgbuf.alloc(16);
    c->cgpart.alloc(5 * DOT_BLOCKS);
    HIPCHK(hipHostMalloc((void**)&c->hpin, 64, hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&c->hcg, 2 * CGS_N * sizeof(double), hipHostMallocDefault));
    for (int k = 0; k < 2; ++k) HIPCHK(hipEventCreateWithFlags(&c->cgev[k], hipEventDisableTiming));
    HIPCHK(hipDeviceSynchronize());
    *out = c.release();
  });
}

int stk_destroy(stk_ctx* ctx) {
  return guard([&] {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->s);
    for (hipEvent_t e : ctx->timer_ev) (void)hipEventDestroy(e);
    if (ctx->hpin) (void)hipHostFree(ctx->hpin);
    if (ctx->hcg) (void)hipHostFree(ctx->hcg);
    for (int k = 0; k < 2; ++k)
      if (ctx->cgev[k]) (void)hipEventDestroy(ctx->cgev[k]);
    delete ctx;
  });
}

int stk_sizes(const stk_ctx* ctx, int level, int64_t* n_p2, int64_t* n_p1) {
  return guard([&] {
    check_level(const_cast<stk_ctx*>(ctx), level);
    if (n_p2) *n_p2 = ctx->lv[level]->h.n2;
    if (n_p1) *n_p1 = ctx->lv[level]->h.n1;
  });
}

int stk_coords(const stk_ctx* ctx, int level, int which, double* xyz, uint8_t* flags) {
  return guard([&] {
    check_level(const_cast<stk_ctx*>(ctx), level);
    REQUIRE(which == 1 || which == 2, "which must be 1 (P1) or 2 (P2)");
    level_coords(ctx->mm, ctx->top, ctx->lv[level]->h, which, xyz, flags);
  });
}

int stk_set_fields(stk_ctx* ctx, const double* eta_p1, const double* lnrho_p1, const stk_solver_params* params) {
  return guard([&] {
    REQUIRE(ctx && eta_p1, "null argument");
    configure_viscosity_levels(*ctx, -1);
    set_fields_internal(*ctx, eta_p1, lnrho_p1, params);
  });
}

int stk_set_log_viscosity(stk_ctx* ctx, const double* m_p1, const double* lnrho_p1, const stk_solver_params* params) {
  return guard([&] {
    REQUIRE(ctx && m_p1, "null argument");
    configure_viscosity_levels(*ctx, -1);
    LevelData& F = ctx->at(ctx->L());
    F.eta.alloc(F.h.n1);
    vexp(m_p1, F.eta.p, F.h.n1, ctx->s);
    set_fields_internal(*ctx, F.eta.p, lnrho_p1, params);
  });
}

int stk_set_temperature_viscosity(stk_ctx* ctx, const double* T_p2, const double* lnrho_p1, const double* eta_base,
                                  int n_base, double E_A, double V_A, int l_eta, const stk_solver_params* params) {
  return guard([&] {
    REQUIRE(ctx && T_p2 && eta_base, "null argument");
    set_temperature_viscosity_internal(*ctx, T_p2, lnrho_p1, eta_base, n_base, E_A, V_A, l_eta, params);
  });
}

int stk_rhs_buoyancy(stk_ctx* ctx, const double* T_p2, double scale, double* f_u) {
  return guard([&] {
    REQUIRE(ctx && T_p2 && f_u, "null argument");
    LevelData& F = ctx->at(ctx->L());
    vfill<double>(f_u, 0.0, 3 * F.h.n2, ctx->s);
    launch_rhs(F.d, T_p2, scale, f_u, ctx->s);
    HIPCHK(hipGetLastError());
  });
}

#define PREC_DISPATCH(prec, CALL64, CALL32)                       \
  do {                                                            \
    if ((prec) == 64) { CALL64; }                                 \
    else if ((prec) == 32) { CALL32; }                            \
    else throw StkError(STK_EINVAL, "prec must be 32 or 64");     \
  } while (0)

int stk_apply_A(stk_ctx* ctx, int level, int prec, const void* x, void* y, int bc) {
  return guard([&] {
    need_ready(ctx);
    check_level(ctx, level);
    REQUIRE(x && y, "null vector");
    PREC_DISPATCH(prec, applyA<double>(*ctx, level, (const double*)x, (double*)y, bc & 3),
                  applyA<float>(*ctx, level, (const float*)x, (float*)y, bc & 3));
    HIPCHK(hipGetLastError());
  });
}

int stk_apply_A_noalloc(stk_ctx* ctx, int level, int prec, const void* x, void* y, int bc) {
  return guard([&] {
    need_ready(ctx);
    check_level(ctx, level);
    REQUIRE(x && y, "null vector");
    REQUIRE(prec == 32 || prec == 64, "prec must be 32 or 64");
    static_assert(NOALLOC_SCRATCH_BYTES == (size_t)STK_NOALLOC_SCRATCH_BYTES, "scratch size mismatch");
    LevelData& L = ctx->at(level);
    const size_t rb = prec == 64 ? sizeof(double) : sizeof(float);
    const size_t n2s = L.d.elemwise ? 0 : (size_t)3 * L.d.nmacro * L.d.sw.nsh2;
    const size_t n1s = L.d.elemwise ? 0 : (size_t)L.d.nmacro * L.d.sw.nsh1;
    const size_t off1 = (n2s * rb + 255) & ~(size_t)255;
    const size_t need = off1 + n1s * rb;
    REQUIRE(need <= NOALLOC_SCRATCH_BYTES,
            "level too large for the allocation-free A-apply: its slots need " + std::to_string(need) +
                " bytes, the fixed scratch holds " + std::to_string(NOALLOC_SCRATCH_BYTES));
    unsigned char* base = static_cast<unsigned char*>(noalloc_scratch(ctx->device));
    REQUIRE(base, "fixed scratch not initialised on this device");
    PREC_DISPATCH(prec,
                  launch_stokes<double>(F_A, L.d, L.bc, (const double*)x, nullptr, L.etap<double>(), nullptr,
                                        (double*)y, nullptr, (double*)base, (double*)(base + off1), bc & 3, ctx->s),
                  launch_stokes<float>(F_A, L.d, L.bc, (const float*)x, nullptr, L.etap<float>(), nullptr,
                                       (float*)y, nullptr, (float*)base, (float*)(base + off1), bc & 3, ctx->s));
    HIPCHK(hipGetLastError());
  });
}

int stk_apply_B(stk_ctx* ctx, int level, int prec, const void* u, void* q, int with_C, int bc) {
  return guard([&] {
    need_ready(ctx);
    check_level(ctx, level);
    REQUIRE(u && q, "null vector");
    PREC_DISPATCH(prec, applyB<double>(*ctx, level, (const double*)u, (double*)q, with_C != 0, bc & 1),
                  applyB<float>(*ctx, level, (const float*)u, (float*)q, with_C != 0, bc & 1));
    HIPCHK(hipGetLastError());
  });
}

int stk_apply_Bt(stk_ctx* ctx, int level, int prec, const void* p, void* y, int with_Ct, int bc) {
  return guard([&] {
    need_ready(ctx);
    check_level(ctx, level);
    REQUIRE(p && y, "null vector");
    PREC_DISPATCH(prec, applyBt<double>(*ctx, level, (const double*)p, (double*)y, with_Ct != 0, bc & 2),
                  applyBt<float>(*ctx, level, (const float*)p, (float*)y, with_Ct != 0, bc & 2));
    HIPCHK(hipGetLastError());
  });
}

int stk_apply_K(stk_ctx* ctx, int prec, const void* u, const void* p, void* yu, void* yp, int transpose, int bc) {
  return guard([&] {
    need_ready(ctx);
    REQUIRE(u && p && yu && yp, "null vector");
    PREC_DISPATCH(prec,
                  applyK<double>(*ctx, (const double*)u, (const double*)p, (double*)yu, (double*)yp, transpose != 0, bc & 3),
                  applyK<float>(*ctx, (const float*)u, (const float*)p, (float*)yu, (float*)yp, transpose != 0, bc & 3));
    HIPCHK(hipGetLastError());
  });
}

int stk_apply_mass(stk_ctx* ctx, int level, int prec, const void* p, void* q) {
  return guard([&] {
    need_ready(ctx);
    check_level(ctx, level);
    REQUIRE(p && q, "null vector");
    PREC_DISPATCH(prec, applyMass<double>(*ctx, level, (const double*)p, (double*)q),
                  applyMass<float>(*ctx, level, (const float*)p, (float*)q));
    HIPCHK(hipGetLastError());
  });
}

int stk_apply_vmass(stk_ctx* ctx, int prec, double a, const void* u, void* y, int bc) {
  return guard([&] {
    need_ready(ctx);
    REQUIRE(u && y, "null vector");
    REQUIRE(a > 0 && std::isfinite(a), "a must be positive");
    LevelData& L = ctx->at(ctx->L());
    PREC_DISPATCH(prec,
                  (launch_vmass<double>(L.d, ctx->vrule, L.etap<double>(), a * a, (const double*)u, (double*)y, false,
                                        bc & BCM_IN, ctx->s),
                   (bc & BCM_OUT) ? launch_project<double>(L.bc, L.h.n2, (double*)y, ctx->s) : (void)0),
                  (launch_vmass<float>(L.d, ctx->vrule, L.etap<float>(), (float)(a * a), (const float*)u, (float*)y,
                                       false, bc & BCM_IN, ctx->s),
                   (bc & BCM_OUT) ? launch_project<float>(L.bc, L.h.n2, (float*)y, ctx->s) : (void)0));
    HIPCHK(hipGetLastError());
  });
}

int stk_apply_poisson(stk_ctx* ctx, int level, int prec, double a, const void* p, void* q) {
  return guard([&] {
    need_ready(ctx);
    check_level(ctx, level);
    REQUIRE(p && q, "null vector");
    REQUIRE(a > 0 && std::isfinite(a), "a must be positive");
    const LevelData::PoissonSet& P = poisson_set(*ctx, level, a * a);
    PREC_DISPATCH(prec, apply_poisson<double>(*ctx, level, P, (const double*)p, (double*)q),
                  apply_poisson<float>(*ctx, level, P, (const float*)p, (float*)q));
    HIPCHK(hipGetLastError());
  });
}

int stk_p1_transfer(stk_ctx* ctx, int level, int prec, int restrict_, const void* in, void* out) {
  return guard([&] {
    REQUIRE(ctx && in && out, "null argument");
    check_level(ctx, level);
    REQUIRE(level > ctx->lmin(), "P1 transfer needs level > min_level");
    LevelData &C = ctx->at(level - 1), &F = ctx->at(level);
    if (restrict_)
      PREC_DISPATCH(prec, launch_p1_restrict<double>(C.d, F.d, (const double*)in, (double*)out, ctx->s),
                    launch_p1_restrict<float>(C.d, F.d, (const float*)in, (float*)out, ctx->s));
    else
      PREC_DISPATCH(prec, launch_p1_prolong<double>(C.d, F.d, (const double*)in, (double*)out, ctx->s),
                    launch_p1_prolong<float>(C.d, F.d, (const float*)in, (float*)out, ctx->s));
    HIPCHK(hipGetLastError());
  });
}

int stk_diag_A(stk_ctx* ctx, int level, double* d) {
  return guard([&] {
    need_ready(ctx);
    check_level(ctx, level);
    REQUIRE(d, "null vector");
    LevelData& L = ctx->at(level);
    vfill<double>(d, 0.0, 3 * L.h.n2, ctx->s);
    if (L.d.qpv) launch_elem_diag(L.d, L.eta.p, d, ctx->s);
    else launch_diag<double>(L.d, L.eta.p, d, ctx->s);
    HIPCHK(hipGetLastError());
  });
}

int stk_cheb_bounds(stk_ctx* ctx, int level, double* lo, double* hi) {
  return guard([&] {
    need_ready(ctx);
    check_level(ctx, level);
    if (lo) *lo = ctx->at(level).lo;
    if (hi) *hi = ctx->at(level).hi;
  });
}

int stk_set_cheb_bounds(stk_ctx* ctx, int level, double lo, double hi) {
  return guard([&] {
    check_level(ctx, level);
    REQUIRE(lo > 0 && hi > lo, "need 0 < lo < hi");
    ctx->at(level).lo = lo;
    ctx->at(level).hi = hi;
    ctx->at(level).bounds_set = true;
  });
}

int stk_smooth(stk_ctx* ctx, int level, int prec, const void* b, void* x, int degree, int steps) {
  return guard([&] {
    need_ready(ctx);
    check_level(ctx, level);
    REQUIRE(b && x, "null vector");
    REQUIRE(degree >= 1 && steps >= 1, "degree and steps must be >= 1");
    REQUIRE(ctx->at(level).hi > 0, "no Chebyshev bounds on this level");
    PREC_DISPATCH(prec, chebyshev<double>(*ctx, level, (const double*)b, (double*)x, steps, degree, false),
                  chebyshev<float>(*ctx, level, (const float*)b, (float*)x, steps, degree, false));
    HIPCHK(hipGetLastError());
  });
}

int stk_prolong(stk_ctx* ctx, int level, int prec, const void* ec, void* ef, int add) {
  return guard([&] {
    REQUIRE(ctx && ec && ef, "null argument");
    check_level(ctx, level);
    REQUIRE(level > ctx->lmin(), "prolongation needs level > min_level");
    REQUIRE(add == 0 || add == 1, "add must be 0 or 1");
    LevelData &C = ctx->at(level - 1), &F = ctx->at(level);
    if (add)
      PREC_DISPATCH(prec, launch_prolong_add<double>(C.d, F.d, (const double*)ec, (double*)ef, BCM_OUT, ctx->s),
                    launch_prolong_add<float>(C.d, F.d, (const float*)ec, (float*)ef, BCM_OUT, ctx->s));
    else
      PREC_DISPATCH(prec, launch_prolong<double>(C.d, F.d, (const double*)ec, (double*)ef, BCM_OUT, ctx->s),
                    launch_prolong<float>(C.d, F.d, (const float*)ec, (float*)ef, BCM_OUT, ctx->s));
    HIPCHK(hipGetLastError());
  });
}

int stk_restrict(stk_ctx* ctx, int level, int prec, const void* rf, const void* tf, void* rc) {
  return guard([&] {
    REQUIRE(ctx && rf && rc, "null argument");
    check_level(ctx, level);
    REQUIRE(level > ctx->lmin(), "restriction needs level > min_level");
    LevelData &C = ctx->at(level - 1), &F = ctx->at(level);
    const long long nc = 3 * C.h.n2;
    if (tf)
      PREC_DISPATCH(prec,
                    (vfill<double>((double*)rc, 0.0, nc, ctx->s),
                     launch_restrict_diff<double>(C.d, F.d, (const double*)rf, (const double*)tf, (double*)rc,
                                                  BCM_IN | BCM_OUT, ctx->s)),
                    (vfill<float>((float*)rc, 0.f, nc, ctx->s),
                     launch_restrict_diff<float>(C.d, F.d, (const float*)rf, (const float*)tf, (float*)rc,
                                                 BCM_IN | BCM_OUT, ctx->s)));
    else
      PREC_DISPATCH(prec,
                    (vfill<double>((double*)rc, 0.0, nc, ctx->s),
                     launch_restrict<double>(C.d, F.d, (const double*)rf, (double*)rc, BCM_OUT, ctx->s)),
                    (vfill<float>((float*)rc, 0.f, nc, ctx->s),
                     launch_restrict<float>(C.d, F.d, (const float*)rf, (float*)rc, BCM_OUT, ctx->s)));
    HIPCHK(hipGetLastError());
  });
}

int stk_vcycle(stk_ctx* ctx, const stk_solver_params* params, int prec, const void* b, void* x, int which) {
  return guard([&] {
    need_ready(ctx);
    check_params(params);
    REQUIRE(b && x, "null vector");
    ctx->par = *params;
    const int st = which == 0 ? params->m_A : params->m_V, dg = which == 0 ? params->deg_A : params->deg_V;
    PREC_DISPATCH(prec, vcycle<double>(*ctx, ctx->L(), (const double*)b, (double*)x, st, dg),
                  vcycle<float>(*ctx, ctx->L(), (const float*)b, (float*)x, st, dg));
    HIPCHK(hipGetLastError());
  });
}

static int solve_common(stk_ctx* ctx, const stk_solver_params* params, const double* f_u, const double* g_p,
                        const double* u_dir, double* u, double* p, stk_report* rep, bool transpose) {
  int status = STK_OK;
  int rc = guard([&] {
    need_ready(ctx);
    check_params(params);
    REQUIRE(f_u && u && p, "null vector");
    ctx->par = *params;
    stk_report local{};
    ctx->rep = &local;
    Ctx& c = *ctx;
    const int l = c.L();
    LevelData& F = c.at(l);
    const long long N = 3 * F.h.n2, n1 = F.h.n1;
    HIPCHK(hipStreamSynchronize(c.s));
    auto t0 = std::chrono::steady_clock::now();
    double* bu = F.pool<double>().get(W_F2, N, c.s);
    double* bp = F.ppool<double>().get(Q_F2, n1, c.s);
    double* ud = F.pool<double>().get(W_F3, N, c.s);
    vcopy<double>(f_u, bu, N, c.s);
    if (g_p) vcopy<double>(g_p, bp, n1, c.s);
    else vfill<double>(bp, 0.0, n1, c.s);
    const bool have_ud = u_dir != nullptr && F.bc.ndir > 0;
    if (have_ud) {
      // u_D restricted to Dirichlet nodes: ud = u_dir - P u_dir
      vcopy<double>(u_dir, ud, N, c.s);
      double* t = F.pool<double>().get(W_U0, N, c.s);
      vcopy<double>(u_dir, t, N, c.s);
      launch_project<double>(BcDev{F.bc.ndir, 0, F.bc.dir, nullptr, nullptr, nullptr}, F.h.n2, t, c.s);
      vaxpy<double>(-1.0, t, ud, N, c.s);
      // b_u -= A u_D, b_p -= Bbar u_D (or B for the transpose)
      double* tp = F.ppool<double>().get(Q_F3, n1, c.s);
      applyA<double>(c, l, ud, t, BCM_OUT);
      vaxpy<double>(-1.0, t, bu, N, c.s);
      applyB<double>(c, l, ud, tp, c.has_rho && !transpose, 0);
      vaxpy<double>(-1.0, tp, bp, n1, c.s);
    }
    FgmresOut fo = fgmres(c, bu, bp, u, p, transpose, params->initial_guess == 1);
    if (have_ud) vaxpy<double>(1.0, ud, u, N, c.s);
    HIPCHK(hipStreamSynchronize(c.s));
    HIPCHK(hipGetLastError());
    auto t1 = std::chrono::steady_clock::now();
    local.iterations = fo.its;
    local.initial_residual = fo.r0;
    local.abs_residual = fo.rfin;
    local.rel_residual = fo.r0 > 0 ? fo.rfin / fo.r0 : 0.0;
    local.seconds = std::chrono::duration<double>(t1 - t0).count();
    ctx->rep = nullptr;
    if (rep) *rep = local;
    if (!fo.converged) status = STK_ENOCONV;
  });
  if (ctx) ctx->rep = nullptr;
  if (rc != STK_OK) return rc;
  if (status == STK_ENOCONV) g_err = "FGMRES reached max_outer before the tolerance";
  return status;
}

int stk_precondition(stk_ctx* ctx, const stk_solver_params* params, const double* ru, const double* rp, double* zu,
                     double* zp, int transpose) {
  return guard([&] {
    need_ready(ctx);
    check_params(params);
    REQUIRE(ru && rp && zu && zp, "null vector");
    ctx->par = *params;
    LevelData& F = ctx->at(ctx->L());
    const long long N = 3 * F.h.n2, n1 = F.h.n1;
    double* v = F.pool<double>().get(W_PC0, N + n1, ctx->s);
    double* z = F.pool<double>().get(W_PC1, N + n1, ctx->s);
    vcopy<double>(ru, v, N, ctx->s);
    vcopy<double>(rp, v + N, n1, ctx->s);
    precondition(*ctx, v, z, transpose != 0);
    vcopy<double>(z, zu, N, ctx->s);
    vcopy<double>(z + N, zp, n1, ctx->s);
    HIPCHK(hipStreamSynchronize(ctx->s));
    HIPCHK(hipGetLastError());
  });
}

int stk_solve(stk_ctx* ctx, const stk_solver_params* params, const double* f_u, const double* g_p,
              const double* u_dirichlet, double* u, double* p, stk_report* rep) {
  return solve_common(ctx, params, f_u, g_p, u_dirichlet, u, p, rep, false);
}

int stk_solve_adjoint(stk_ctx* ctx, const stk_solver_params* params, const double* ju, const double* jp, double* lu,
                      double* lp, stk_report* rep) {
  return solve_common(ctx, params, ju, jp, nullptr, lu, lp, rep, true);
}

int stk_gradient(stk_ctx* ctx, const double* u, const double* lu, double scale, double* g_m, double* g_T) {
  return guard([&] {
    need_ready(ctx);
    REQUIRE(u && lu && g_m && g_T, "null vector");
    LevelData& F = ctx->at(ctx->L());
    vfill<double>(g_m, 0.0, F.h.n1, ctx->s);
    vfill<double>(g_T, 0.0, F.h.n2, ctx->s);
    launch_gradient(F.d, F.eta.p, u, lu, g_m, g_T, scale, ctx->s);
    HIPCHK(hipGetLastError());
  });
}

int stk_time_apply_A(stk_ctx* ctx, int level, int prec, const void* x, void* y, int reps, double* ms_apply,
                     double* ms_kernel) {
  return guard([&] {
    need_ready(ctx);
    check_level(ctx, level);
    REQUIRE(x && y && ms_apply && reps >= 1, "bad argument");
    REQUIRE(prec == 32 || prec == 64, "prec must be 32 or 64");
    LevelData& L = ctx->at(level);
    hipEvent_t e0, e1, e2;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventCreate(&e2));
    // whole operator: sweep + gather + projection
    HIPCHK(hipEventRecord(e0, ctx->s));
    for (int i = 0; i < reps; ++i) {
      if (prec == 64) applyA<double>(*ctx, level, (const double*)x, (double*)y, BCM_IN | BCM_OUT);
      else applyA<float>(*ctx, level, (const float*)x, (float*)y, BCM_IN | BCM_OUT);
    }
    HIPCHK(hipEventRecord(e1, ctx->s));
    // the sweep kernel alone (gather lists emptied)
    LevelDev d = L.d;
    d.g2.nnodes = 0;
    BcDev nobc{};
    for (int i = 0; i < reps; ++i) {
      if (prec == 64)
        launch_stokes<double>(F_A, d, nobc, (const double*)x, nullptr, L.eta.p, nullptr, (double*)y, nullptr,
                              L.sl2<double>(), L.sl1<double>(), BCM_IN, ctx->s);
      else
        launch_stokes<float>(F_A, d, nobc, (const float*)x, nullptr, L.etaf.p, nullptr, (float*)y, nullptr,
                             L.sl2<float>(), L.sl1<float>(), BCM_IN, ctx->s);
    }
    HIPCHK(hipEventRecord(e2, ctx->s));
    HIPCHK(hipEventSynchronize(e2));
    float a = 0, b = 0;
    HIPCHK(hipEventElapsedTime(&a, e0, e1));
    HIPCHK(hipEventElapsedTime(&b, e1, e2));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipEventDestroy(e2);
    *ms_apply = a / reps;
    if (ms_kernel) *ms_kernel = b / reps;
  });
}

// ---- temperature step ---------------------------------------------------------------
void stk_temp_default_params(stk_temp_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->tau1 = 1e-3;
  p->tau0 = 1e-3;
  p->k = 1.0;
  p->Pe = 1.0;
  p->Cp = 1.0;
  p->Ra = 1.0;
  p->T_in = 1.0;
  p->T_out = 0.0;
  p->tol_abs = 1e-10;
  p->tol_cg = 1e-12;
  p->restart = 30;
  p->max_outer = 300;
  p->max_cg = 5000;
  p->stored_S = 1;
}

int stk_temp_apply(stk_ctx* ctx, const stk_temp_params* p, int mode, const double* u_star, const double* lnrho,
                   const double* x, double* y) {
  return guard([&] {
    REQUIRE(ctx && ctx->lv.size() > 0, "null context");
    check_temp_params(p);
    REQUIRE(mode == STK_TEMP_APPLY || mode == STK_TEMP_SYM || mode == STK_TEMP_DIAG || mode == STK_TEMP_SYM_STORED,
            "unknown mode");
    REQUIRE(y && (x || mode == STK_TEMP_DIAG), "null vector");
    REQUIRE(x != y, "x and y must be distinct buffers");
    const TempCoef tc = temp_coef(*p);
    if (mode == STK_TEMP_SYM_STORED) {
      REQUIRE(temp_build_smat(*ctx, tc, lnrho, true), "not enough free device memory for the stored matrices");
      launch_temp_sapply(ctx->at(ctx->L()).d, ctx->temp.smat.p, x, y, ctx->s);
    } else {
      const int m = mode == STK_TEMP_APPLY ? TM_APPLY : (mode == STK_TEMP_SYM ? TM_SYM : TM_DIAG);
      temp_apply(*ctx, tc, m, x, mode == STK_TEMP_APPLY ? u_star : nullptr, lnrho, y);
    }
    HIPCHK(hipGetLastError());
  });
}

int stk_temp_rhs(stk_ctx* ctx, const stk_temp_params* p, const double* u_star, const double* lnrho, const double* eta,
                 const double* That_n, const double* That_nm1, double* b) {
  return guard([&] {
    REQUIRE(ctx && ctx->lv.size() > 0, "null context");
    check_temp_params(p);
    REQUIRE(That_n && That_nm1 && b, "null vector");
    REQUIRE(!u_star || eta, "eta is needed with a velocity");
    LevelData& L = ctx->at(ctx->L());
    launch_temp(L.d, ctx->vrule, temp_coef(*p), TM_RHS, nullptr, u_star, lnrho, eta, That_n, That_nm1, b, ctx->s);
    HIPCHK(hipGetLastError());
  });
}

int stk_mmoc(stk_ctx* ctx, const double* F, const double* u_new, const double* u_old, double tau, double* out) {
  return guard([&] {
    REQUIRE(ctx && ctx->lv.size() > 0, "null context");
    REQUIRE(F && u_new && u_old && out, "null vector");
    REQUIRE(F != out, "F and out must be distinct buffers");
    REQUIRE(std::isfinite(tau) && tau >= 0, "tau must be finite and >= 0");
    setup_temp(*ctx);
    launch_mmoc(ctx->at(ctx->L()).d, ctx->temp.loc, F, u_new, u_old, tau, out, ctx->s);
    HIPCHK(hipGetLastError());
  });
}

int stk_temp_solve(stk_ctx* ctx, const stk_temp_params* p, const double* u_star, const double* lnrho,
                   const double* b, const double* T_init, double* T, stk_temp_report* rep) {
  return guard([&] {
    REQUIRE(ctx && ctx->lv.size() > 0, "null context");
    check_temp_params(p);
    REQUIRE(b && T, "null vector");
    REQUIRE(T != b && T_init != b, "T must not alias b");
    if (rep) std::memset(rep, 0, sizeof(*rep));
    const auto t0 = std::chrono::steady_clock::now();
    temp_solve(*ctx, *p, u_star, lnrho, b, T_init, T, rep);
    if (rep) rep->ms_solve = ms_since(t0);
  });
}

int stk_temperature_step(stk_ctx* ctx, const stk_temp_params* p, const double* T_n, const double* T_nm1,
                         const double* u_n, const double* u_nm1, const double* lnrho, const double* eta,
                         double* T_np1, double* That_n, double* That_nm1, stk_temp_report* rep) {
  return guard([&] {
    REQUIRE(ctx && ctx->lv.size() > 0, "null context");
    temperature_step_internal(*ctx, p, T_n, T_nm1, u_n, u_nm1, lnrho, eta, T_np1, That_n, That_nm1, rep);
  });
}

int stk_coupled_step(stk_ctx* ctx, const stk_solver_params* sp, const stk_temp_params* tp, const double* eta_base,
                     int n_base, double E_A, double V_A, int l_eta, double buoyancy_scale, const double* lnrho,
                     const double* T_n, const double* T_nm1, const double* u_n, const double* u_nm1,
                     const double* p_n, double* T_np1, double* u_np1, double* p_np1, stk_temp_report* trep,
                     stk_report* srep) {
  const int rc = guard([&] {
    REQUIRE(ctx && ctx->lv.size() > 0, "null context");
    REQUIRE(sp && eta_base && u_np1 && p_np1, "null argument");
    REQUIRE(std::isfinite(buoyancy_scale), "buoyancy_scale must be finite");
    check_temp_params(tp);
    REQUIRE(T_n && T_nm1, "null vector");
    Ctx& c = *ctx;
    const long long n2 = n2of(c, c.L());
    // T* = T^n + (T^n - T^{n-1}) tau^{n+1} / tau^n and the viscosity at it
    c.temp.tstar.alloc((size_t)n2);
    const double q = tp->tau1 / tp->tau0;
    vcopy<double>(T_n, c.temp.tstar.p, n2, c.s);
    vaxpby<double>(-q, T_nm1, 1.0 + q, c.temp.tstar.p, n2, c.s);
    set_temperature_viscosity_internal(c, c.temp.tstar.p, lnrho, eta_base, n_base, E_A, V_A, l_eta, sp);
    temperature_step_internal(c, tp, T_n, T_nm1, u_n, u_nm1, lnrho, c.at(c.L()).eta.p, T_np1, nullptr, nullptr,
                              trep);
    // the Stokes fields at T^{n+1} and the buoyancy of T^{n+1}
    set_temperature_viscosity_internal(c, T_np1, lnrho, eta_base, n_base, E_A, V_A, l_eta, sp);
    LevelData& F = c.at(c.L());
    c.temp.fbuf.alloc((size_t)3 * n2);
    vfill<double>(c.temp.fbuf.p, 0.0, 3 * n2, c.s);
    launch_rhs(F.d, T_np1, buoyancy_scale, c.temp.fbuf.p, c.s);
    if (sp->initial_guess == 1) {
      // the Stokes solve starts from the step's previous solution
      REQUIRE(u_np1 != u_n && (!p_n || p_np1 != p_n), "outputs must not alias u_n, p_n");
      vcopy<double>(u_n, u_np1, 3 * n2, c.s);
      if (p_n) vcopy<double>(p_n, p_np1, n1of(c, c.L()), c.s);
      else vfill<double>(p_np1, 0.0, n1of(c, c.L()), c.s);
    }
    HIPCHK(hipGetLastError());
  });
  if (rc != STK_OK) return rc;
  return solve_common(ctx, sp, ctx->temp.fbuf.p, nullptr, nullptr, u_np1, p_np1, srep, false);
}

int stk_kernel_timer(stk_ctx* ctx, int enable, double* ms_total, int* launches) {
  return guard([&] {
    REQUIRE(ctx, "null context");
    if (enable) {
      while (ctx->timer_ev.size() < 128) {   // 64 pairs up front; more are made on demand
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        ctx->timer_ev.push_back(e);
      }
      ctx->timer_on = true;
      ctx->timer_n = 0;
      return;
    }
    ctx->timer_on = false;
    double tot = 0;
    for (int i = 0; i < ctx->timer_n; ++i) {
      HIPCHK(hipEventSynchronize(ctx->timer_ev[2 * i + 1]));
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, ctx->timer_ev[2 * i], ctx->timer_ev[2 * i + 1]));
      tot += ms;
    }
    if (ms_total) *ms_total = tot;
    if (launches) *launches = ctx->timer_n;
    ctx->timer_n = 0;
  });
}

}  // extern "C"
