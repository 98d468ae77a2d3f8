// SBCI1 driver (Algorithm 1 with Supplementary Sections S1.1-S1.5) and the
// block Davidson baseline, both on the device sigma of sigma.hip and the
// vector passes of vec.hip.  Per SBCI step the host reads back at most ~30
// FP64 scalars, solves the 2x2 or 3x3 Ritz problem and launches the next
// pass; vectors never leave the GPU.
//
// Step of root alpha (t counts steps inside the current segment):
//   sigma:   Z = H z                                   (Eq. S32)
//   dots:    x.Z, y.Z, z.Z                            (H on the right vector)
//   Ritz:    t = 0: 2x2 V_0 (Eqs. S10-S24), b = 1, c, k
//            t > 0: 3x3 V_t (Eqs. S33-S55), b, c, k
//   update:  y, Y, x, X, z' and the next preconditioned residual in one
//            pass (Eqs. S56-S60 and S31), plus the next Gram dots
//   test:    dE < eps0 and |z'| < r0 (Eq. S61), else restart on S62a-c or
//            after max_cycle steps (Section S1.5)
//   deflate: z <- z - sum x_c (x_c . z)                (Eq. S31)
// A restart divides x, X by |x| lazily: the next update pass applies the
// scale, and the host rescales the dots it already has.
//
// Precision form: with opt.precision = SBCI_F32 or SBCI_BF16 each root first
// runs with FP32 vectors and a low-precision sigma (all reductions, the Ritz
// problem, the restart tests and the deflation stay FP64).  SBCI_BF16 starts
// with the BF16-MFMA sigma and moves to the FP32 sigma at bf16_eps0 /
// bf16_r0; the FP32 phase ends at mix_eps0 / mix_r0 (either phase also ends
// after mix_stall steps without an energy decrease).  Each hand-over
// recomputes X = H x with the next sigma and starts a new segment; the last
// one promotes x to FP64, and FP64 steps refine it to eps0 / r0.
#include "internal.h"
#include "ritz.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

namespace sbci {

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

enum Slot { X_ = 0, XX_ = 1, Y_ = 2, YY_ = 3, ZA_ = 4, ZB_ = 5, Z_ = 6, NV = 7 };

}  // namespace

struct Solver {
  sbci_opts o{};
  int nroots = 0;
  int64_t n = 0;
  double *v64[NV] = {};
  float *v32[NV] = {};
  std::vector<double *> xc64;
  std::vector<float *> xc32;
  std::vector<double> Ec;
  double *red = nullptr;  // device results: [0,32) update, [32,36) deflate, [36,40) dots_xyz, [40,64) misc
  double h1[32] = {}, h2[4] = {}, h3[4] = {};
  // per-root state
  int alpha = 0, seg = 0, t = 0, steps_root = 0;
  int phase = SBCI_F64;   // precision of the running phase
  double E = 0, sx = 1;
  bool seg_start = true;
  int zc = ZA_, zn = ZB_;
  Ritz last;
  int stall = 0;
  double bestE = 0;
  double last_dz = 0;     // |z'| of the latest step (the residual of a converged root)
  bool done = false;
  bool any_noconv = false;
  // report
  sbci_report rep{};
  double t0 = 0;
  std::vector<double> resid;
  size_t alloc_bytes = 0;

  template <typename T>
  T *vec(int slot);
  template <typename T>
  std::vector<T *> &xcs();
};

template <>
double *Solver::vec<double>(int s) { return v64[s]; }
template <>
float *Solver::vec<float>(int s) { return v32[s]; }
template <>
std::vector<double *> &Solver::xcs<double>() { return xc64; }
template <>
std::vector<float *> &Solver::xcs<float>() { return xc32; }

namespace {

double precond_shift(const Solver &S, double Enew) { return S.alpha == 0 ? Enew : S.Ec[0]; }

int read_back(sbci_ctx *ctx, Solver &S, int which) {
  // which: bit0 update slots, bit1 deflate, bit2 dots_xyz
  if (which & 1) SBCI_HIP(hipMemcpyAsync(S.h1, S.red, sizeof(double) * 32, hipMemcpyDeviceToHost, ctx->stream));
  if (which & 2) SBCI_HIP(hipMemcpyAsync(S.h2, S.red + 32, sizeof(double) * 4, hipMemcpyDeviceToHost, ctx->stream));
  if (which & 4) SBCI_HIP(hipMemcpyAsync(S.h3, S.red + 36, sizeof(double) * 4, hipMemcpyDeviceToHost, ctx->stream));
  SBCI_HIP(hipStreamSynchronize(ctx->stream));
  return SBCI_OK;
}

int alloc_solver(sbci_ctx *ctx, Solver &S, bool need32) {
  const int64_t n = ctx->ndet;
  for (int i = 0; i < NV; ++i) {
    if (!S.v64[i]) {
      SBCI_HIP(hipMalloc(&S.v64[i], sizeof(double) * n));
      SBCI_HIP(hipMemsetAsync(S.v64[i], 0, sizeof(double) * n, ctx->stream));
      S.alloc_bytes += sizeof(double) * n;
    }
    if (need32 && !S.v32[i]) {
      SBCI_HIP(hipMalloc(&S.v32[i], sizeof(float) * n));
      SBCI_HIP(hipMemsetAsync(S.v32[i], 0, sizeof(float) * n, ctx->stream));
      S.alloc_bytes += sizeof(float) * n;
    }
  }
  if (!S.red) {
    SBCI_HIP(hipMalloc(&S.red, sizeof(double) * 64));
    SBCI_HIP(hipMemsetAsync(S.red, 0, sizeof(double) * 64, ctx->stream));
  }
  return SBCI_OK;
}

void record(sbci_ctx *ctx, Solver &S, double Enew, double dE, double dz, double b, double c,
            double k, double xn, int reason) {
  if (!ctx->trace_on) return;
  sbci_step_info r{};
  r.root = S.alpha;
  r.segment = S.seg;
  r.t = S.t;
  r.precision = S.phase;
  r.E = Enew;
  r.dE = dE;
  r.dz = dz;
  r.b = b;
  r.c = c;
  r.k = k;
  r.xnorm = xn;
  r.seconds = now_s() - S.t0;
  r.reason = reason;
  ctx->trace.push_back(r);
}

// Segment start: x, X hold an unnormalised start vector (scale sx pending);
// computes z'0 = (X0 - E x0) and the preconditioned, deflated z0.
template <typename T>
int segment_start(sbci_ctx *ctx, Solver &S, double sx) {
  const int nconv = (int)S.Ec.size();
  UpdateArgs a{};
  a.b = 0;
  a.c = 0;
  a.E = S.E;
  a.inv_norm = 1.0;
  a.E0 = precond_shift(S, S.E);
  a.floor = S.o.precond_floor;
  a.sx = sx;
  a.sy = 0;
  a.read_z = 0;
  a.nconv = nconv;
  a.want_zdots = nconv == 0;
  auto &xc = S.xcs<T>();
  std::vector<const T *> xcp(xc.begin(), xc.end());
  const T *D = std::is_same<T, double>::value ? (const T *)ctx->hdiag : (const T *)ctx->hdiag32;
  SBCI_TRY(update<T>(ctx, S.n, S.vec<T>(X_), S.vec<T>(XX_), S.vec<T>(Y_), S.vec<T>(YY_), nullptr,
                     nullptr, S.vec<T>(S.zc), D, xcp.data(), a, S.red));
  if (nconv > 0) {
    SBCI_TRY(deflate<T>(ctx, S.n, S.vec<T>(S.zc), S.vec<T>(X_), S.vec<T>(Y_), xcp.data(), nconv,
                        S.red + 10, S.red + 32));
    SBCI_TRY(read_back(ctx, S, 3));
  } else {
    SBCI_TRY(read_back(ctx, S, 1));
  }
  S.sx = 1.0;
  S.seg_start = true;
  S.t = 0;
  return SBCI_OK;
}

// Start of a root from x, X (unnormalised, in the running precision) with
// energy S.E: Algorithm 1 line 1 with Eqs. S4-S7, then the segment start.
template <typename T>
int start_root(sbci_ctx *ctx, Solver &S) {
  const int nconv = (int)S.Ec.size();
  auto &xc = S.xcs<T>();
  T *x = S.vec<T>(X_), *X = S.vec<T>(XX_);
  if (nconv > 0) {
    std::vector<const T *> xcp(xc.begin(), xc.end());
    SBCI_TRY(dots<T>(ctx, S.n, x, xcp.data(), nconv, S.red + 40));
    double d[16];
    SBCI_HIP(hipMemcpyAsync(d, S.red + 40, sizeof(double) * nconv, hipMemcpyDeviceToHost, ctx->stream));
    SBCI_HIP(hipStreamSynchronize(ctx->stream));
    double cx[16], cX[16];
    for (int i = 0; i < nconv; ++i) {
      cx[i] = -d[i];
      cX[i] = -S.Ec[i] * d[i];
    }
    SBCI_TRY(lincomb<T>(ctx, S.n, x, xcp.data(), cx, nconv, 1.0));   // Eq. S4
    SBCI_TRY(lincomb<T>(ctx, S.n, X, xcp.data(), cX, nconv, 1.0));   // Eq. S5
  }
  const T *xp[1] = {x};
  SBCI_TRY(dots<T>(ctx, S.n, x, xp, 1, S.red + 40));
  double nxx;
  SBCI_HIP(hipMemcpyAsync(&nxx, S.red + 40, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  SBCI_HIP(hipStreamSynchronize(ctx->stream));
  if (!(nxx > 0) || !std::isfinite(nxx))
    return set_error(SBCI_ENUMERIC, "start vector vanished after projection");
  S.seg = 0;
  S.steps_root = 0;
  S.stall = 0;
  S.bestE = S.E;
  return segment_start<T>(ctx, S, 1.0 / std::sqrt(nxx));  // Eqs. S6-S7 applied lazily
}

template <typename T>
int sigma_phase(sbci_ctx *ctx, Solver &S, const T *c, T *out) {
  if (std::is_same<T, double>::value) {
    S.rep.nsigma_f64 += 1;
    return sigma(ctx, c, out, 1, SBCI_F64);
  }
  S.rep.nsigma_low += 1;
  if (S.phase == SBCI_BF16) S.rep.nsigma_bf16 += 1;
  return sigma(ctx, c, out, 1, S.phase);
}

// BF16 phase -> FP32 phase: X = H x recomputed with the FP32 sigma (the
// carried X holds the BF16 contraction's error) and a new segment starts.
int to_f32(sbci_ctx *ctx, Solver &S) {
  SBCI_TRY(sigma(ctx, S.v32[X_], S.v32[XX_], 1, SBCI_F32));
  S.rep.nsigma_low += 1;
  const float *xp[1] = {S.v32[X_]};
  const float *Xp[1] = {S.v32[XX_]};
  SBCI_TRY(dots<float>(ctx, S.n, S.v32[X_], xp, 1, S.red + 40));
  SBCI_TRY(dots<float>(ctx, S.n, S.v32[X_], Xp, 1, S.red + 41));
  double d[2];
  SBCI_HIP(hipMemcpyAsync(d, S.red + 40, sizeof(double) * 2, hipMemcpyDeviceToHost, ctx->stream));
  SBCI_HIP(hipStreamSynchronize(ctx->stream));
  S.E = d[1] / d[0];
  S.phase = SBCI_F32;
  const int steps = S.steps_root, seg = S.seg;
  SBCI_TRY(start_root<float>(ctx, S));
  S.steps_root = steps;
  S.seg = seg + 1;
  return SBCI_OK;
}

// Promote the low-precision iterate to FP64 and restart there (refinement).
int promote(sbci_ctx *ctx, Solver &S) {
  SBCI_TRY((convert<double, float>(ctx, S.n, S.v64[X_], S.v32[X_], 1.0)));
  SBCI_TRY(sigma(ctx, S.v64[X_], S.v64[XX_], 1, SBCI_F64));
  S.rep.nsigma_f64 += 1;
  const double *xp[1] = {S.v64[X_]};
  const double *Xp[1] = {S.v64[XX_]};
  SBCI_TRY(dots<double>(ctx, S.n, S.v64[X_], xp, 1, S.red + 40));
  SBCI_TRY(dots<double>(ctx, S.n, S.v64[X_], Xp, 1, S.red + 41));
  double d[2];
  SBCI_HIP(hipMemcpyAsync(d, S.red + 40, sizeof(double) * 2, hipMemcpyDeviceToHost, ctx->stream));
  SBCI_HIP(hipStreamSynchronize(ctx->stream));
  S.E = d[1] / d[0];
  S.phase = SBCI_F64;
  int steps = S.steps_root;
  int seg = S.seg;
  SBCI_TRY(start_root<double>(ctx, S));
  S.steps_root = steps;
  S.seg = seg + 1;
  return SBCI_OK;
}

// Finish root alpha in FP64 and prepare the next root's start vector from
// the second Ritz vector of the converging step (Section S1.4).
int finish_root(sbci_ctx *ctx, Solver &S, double xn, bool second_ok) {
  double *xc = nullptr;
  SBCI_HIP(hipMalloc(&xc, sizeof(double) * S.n));
  S.alloc_bytes += sizeof(double) * S.n;
  SBCI_TRY((convert<double, double>(ctx, S.n, xc, S.v64[X_], 1.0 / xn)));
  S.xc64.push_back(xc);
  if (S.o.precision != SBCI_F64) {
    float *x32 = nullptr;
    SBCI_HIP(hipMalloc(&x32, sizeof(float) * S.n));
    S.alloc_bytes += sizeof(float) * S.n;
    SBCI_TRY((convert<float, double>(ctx, S.n, x32, xc, 1.0)));
    S.xc32.push_back(x32);
  }
  const double Enew = S.E;
  S.Ec.push_back(Enew);
  S.rep.resid[std::min(S.alpha, 15)] = S.last_dz;
  S.rep.t_converged[std::min(S.alpha, 15)] = now_s() - S.t0;
  S.rep.nroots_converged = (int)S.Ec.size();
  if ((int)S.Ec.size() >= S.nroots) {
    S.done = true;
    return SBCI_OK;
  }
  if (!second_ok) return set_error(SBCI_ENUMERIC, "no second Ritz vector for the next root");
  // v2 = a_x x_t + a_y y_t + a_z z_t with x_t = x - b y, y_t = y + c z_t
  const double ax = S.last.a2[0], ay = S.last.a2[1], az = S.last.a2[2];
  const double b = S.last.b, c = S.last.c;
  double cf[3] = {ax, ay - ax * b, ay * c + az};
  const double *in1[3] = {S.v64[X_], S.v64[Y_], S.v64[S.zc]};
  const double *in2[3] = {S.v64[XX_], S.v64[YY_], S.v64[Z_]};
  SBCI_TRY(lincomb<double>(ctx, S.n, S.v64[S.zn], in1, cf, 3, 0.0));
  SBCI_TRY(lincomb<double>(ctx, S.n, S.v64[YY_], in2, cf, 3, 0.0));   // in place on Y is elementwise-safe
  std::swap(S.v64[X_], S.v64[S.zn]);
  std::swap(S.v64[XX_], S.v64[YY_]);
  S.E = S.last.E[1];
  S.alpha += 1;
  if (S.o.precision != SBCI_F64) {
    SBCI_TRY((convert<float, double>(ctx, S.n, S.v32[X_], S.v64[X_], 1.0)));
    SBCI_TRY((convert<float, double>(ctx, S.n, S.v32[XX_], S.v64[XX_], 1.0)));
    S.phase = S.o.precision;
    return start_root<float>(ctx, S);
  }
  S.phase = SBCI_F64;
  return start_root<double>(ctx, S);
}

// Restart from the lowest Ritz vector when the update cannot express it
// (vanishing Gram-Schmidt radicand or coefficient).
template <typename T>
int restart_from_ritz(sbci_ctx *ctx, Solver &S, const Ritz &r) {
  double cf[3] = {r.a1[0], S.seg_start ? 0.0 : r.a1[1], r.a1[2]};
  const T *in1[3] = {S.vec<T>(X_), S.vec<T>(Y_), S.vec<T>(S.zc)};
  const T *in2[3] = {S.vec<T>(XX_), S.vec<T>(YY_), S.vec<T>(Z_)};
  // account for the pending scale of x
  cf[0] *= S.sx;
  SBCI_TRY(lincomb<T>(ctx, S.n, S.vec<T>(S.zn), in1, cf, 3, 0.0));
  SBCI_TRY(lincomb<T>(ctx, S.n, S.vec<T>(YY_), in2, cf, 3, 0.0));
  if (std::is_same<T, double>::value) {
    std::swap(S.v64[X_], S.v64[S.zn]);
    std::swap(S.v64[XX_], S.v64[YY_]);
  } else {
    std::swap(S.v32[X_], S.v32[S.zn]);
    std::swap(S.v32[XX_], S.v32[YY_]);
  }
  S.E = r.E[0];
  S.seg += 1;
  S.rep.nrestarts += 1;
  const T *xp[1] = {S.vec<T>(X_)};
  SBCI_TRY(dots<T>(ctx, S.n, S.vec<T>(X_), xp, 1, S.red + 40));
  double nxx;
  SBCI_HIP(hipMemcpyAsync(&nxx, S.red + 40, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  SBCI_HIP(hipStreamSynchronize(ctx->stream));
  return segment_start<T>(ctx, S, 1.0 / std::sqrt(nxx));
}

template <typename T>
int step_t(sbci_ctx *ctx, Solver &S, sbci_step_info *info) {
  const int nconv = (int)S.Ec.size();
  T *z = S.vec<T>(S.zc);
  T *Z = S.vec<T>(Z_);
  SBCI_TRY(sigma_phase<T>(ctx, S, z, Z));                                      // Eq. S32
  SBCI_TRY(dots_xyz<T>(ctx, S.n, S.vec<T>(X_), S.vec<T>(Y_), z, Z, S.red + 36));
  SBCI_TRY(read_back(ctx, S, 4));
  S.steps_root += 1;
  S.rep.nsteps += 1;
  const double sx = S.sx;
  double N[6], Hm[6];
  N[0] = sx * sx * S.h1[1];
  N[1] = sx * S.h1[2];
  N[3] = S.h1[3];
  Hm[0] = sx * sx * S.h1[4];
  Hm[1] = sx * S.h1[5];
  Hm[3] = S.h1[6];
  if (nconv > 0) {
    N[2] = sx * S.h2[0];
    N[4] = S.h2[1];
    N[5] = S.h2[2];
  } else {
    N[2] = sx * S.h1[7];
    N[4] = S.h1[8];
    N[5] = S.h1[9];
  }
  Hm[2] = sx * S.h3[0];
  Hm[4] = S.h3[1];
  Hm[5] = S.h3[2];
  for (int i = 0; i < 6; ++i)
    if (!std::isfinite(N[i]) || !std::isfinite(Hm[i]))
      return set_error(SBCI_ENUMERIC, "non-finite reduction in SBCI step");
  Ritz r = S.seg_start ? ritz_first(N[0], N[2], N[5], Hm[0], Hm[2], Hm[5], S.o.lindep)
                       : ritz_next(N, Hm, S.o.lindep);
  if (!r.rank_ok) {
    if (S.seg_start) {
      // z in span{x} at a segment start: x is already an eigenvector (e.g.
      // N_det = 1) when its residual is below r0; otherwise unrecoverable.
      const double dz0 = std::sqrt(S.h1[0]);
      if (S.phase == SBCI_F64 && dz0 < S.o.r0) {
        S.last_dz = dz0;
        record(ctx, S, S.E, 0.0, dz0, 0.0, 0.0, 1.0, std::sqrt(N[0]), 1);
        if (info) *info = ctx->trace.back();
        return finish_root(ctx, S, std::sqrt(S.h1[1]), false);
      }
      if (S.phase != SBCI_F64) return promote(ctx, S);
      return set_error(SBCI_ENUMERIC, "SBCI: residual direction parallel to x at a segment start");
    }
    record(ctx, S, S.E, NAN, NAN, NAN, NAN, NAN, std::sqrt(N[0]), 6);
    S.rep.nrestarts += 1;
    S.seg += 1;
    if (info) *info = ctx->trace.empty() ? sbci_step_info{} : ctx->trace.back();
    return segment_start<T>(ctx, S, sx / std::sqrt(N[0]) * 1.0);
  }
  if (!r.coef_ok) {
    record(ctx, S, r.E[0], NAN, NAN, NAN, NAN, NAN, NAN, 7);
    if (info) *info = ctx->trace.empty() ? sbci_step_info{} : ctx->trace.back();
    return restart_from_ritz<T>(ctx, S, r);
  }
  const double Enew = r.E[0];
  UpdateArgs a{};
  a.b = r.b;
  a.c = r.c;
  a.E = Enew;
  a.inv_norm = 1.0 / std::fabs(r.k);
  a.E0 = precond_shift(S, Enew);
  a.floor = S.o.precond_floor;
  a.sx = sx;
  a.sy = S.seg_start ? 0 : 1;
  a.read_z = 1;
  a.nconv = nconv;
  a.want_zdots = nconv == 0;
  auto &xc = S.xcs<T>();
  std::vector<const T *> xcp(xc.begin(), xc.end());
  const T *D = std::is_same<T, double>::value ? (const T *)ctx->hdiag : (const T *)ctx->hdiag32;
  SBCI_TRY(update<T>(ctx, S.n, S.vec<T>(X_), S.vec<T>(XX_), S.vec<T>(Y_), S.vec<T>(YY_), z, Z,
                     S.vec<T>(S.zn), D, xcp.data(), a, S.red));
  SBCI_TRY(read_back(ctx, S, 1));
  S.last = r;
  const double dz = std::sqrt(S.h1[0]);
  const double xn = std::sqrt(S.h1[1]);
  const double dE = std::fabs(Enew - S.E);
  S.last_dz = dz;
  if (!std::isfinite(dz) || !std::isfinite(xn) || !std::isfinite(Enew))
    return set_error(SBCI_ENUMERIC, "non-finite residual or norm");
  int reason = 0;
  bool conv = false, promote_now = false;
  const bool low = S.phase != SBCI_F64;
  if (!low && dE < S.o.eps0 && dz < S.o.r0) {
    conv = true;
    reason = 1;
  } else if (low) {
    if (Enew < S.bestE - 1e-15 * std::fabs(S.bestE)) {
      S.bestE = Enew;
      S.stall = 0;
    } else {
      S.stall += 1;
    }
    const bool bf = S.phase == SBCI_BF16;
    const double e0 = bf ? S.o.bf16_eps0 : S.o.mix_eps0, r0 = bf ? S.o.bf16_r0 : S.o.mix_r0;
    if ((dE < e0 && dz < r0) || S.stall >= S.o.mix_stall) {
      promote_now = true;
      reason = 8;
    }
  }
  if (!conv && !promote_now) {
    const bool s62a = S.alpha > 0 && std::fabs(r.b) < S.o.b_th && dE < S.o.eps1;
    const bool s62b = xn < S.o.x_th1 || xn > S.o.x_th2;
    const bool s62c = dz > S.o.r1 && S.t > 0;
    const bool cap = S.t + 1 >= S.o.max_cycle;
    reason = s62a ? 2 : s62b ? 3 : s62c ? 4 : cap ? 5 : 0;
  }
  record(ctx, S, Enew, dE, dz, r.b, r.c, r.k, xn, reason);
  if (info) *info = ctx->trace.empty() ? sbci_step_info{} : ctx->trace.back();
  S.E = Enew;
  if (conv) return finish_root(ctx, S, xn, true);
  if (promote_now) return S.phase == SBCI_BF16 ? to_f32(ctx, S) : promote(ctx, S);
  if (S.steps_root >= S.o.max_steps) {
    S.any_noconv = true;
    if (low) return promote(ctx, S);
    return finish_root(ctx, S, xn, true);
  }
  if (reason >= 2) {
    S.rep.nrestarts += 1;
    S.seg += 1;
    S.t = 0;
    S.seg_start = true;
    S.sx = 1.0 / xn;
  } else {
    S.t += 1;
    S.seg_start = false;
    S.sx = 1.0;
  }
  if (nconv > 0) {
    SBCI_TRY(deflate<T>(ctx, S.n, S.vec<T>(S.zn), S.vec<T>(X_), S.vec<T>(Y_), xcp.data(), nconv,
                        S.red + 10, S.red + 32));
    SBCI_TRY(read_back(ctx, S, 2));
  }
  std::swap(S.zc, S.zn);
  return SBCI_OK;
}

// Section S1.1: the nroots lowest diagonal determinants (ties: lower index).
int lowest_diagonal(sbci_ctx *ctx, int k, std::vector<int64_t> &idx) {
  std::vector<double> D((size_t)ctx->ndet);
  SBCI_HIP(hipMemcpyAsync(D.data(), ctx->hdiag, sizeof(double) * ctx->ndet, hipMemcpyDeviceToHost,
                          ctx->stream));
  SBCI_HIP(hipStreamSynchronize(ctx->stream));
  std::vector<int64_t> order((size_t)ctx->ndet);
  for (int64_t i = 0; i < ctx->ndet; ++i) order[i] = i;
  std::partial_sort(order.begin(), order.begin() + k, order.end(), [&](int64_t a, int64_t b) {
    return D[a] < D[b] || (D[a] == D[b] && a < b);
  });
  idx.assign(order.begin(), order.begin() + k);
  return SBCI_OK;
}

__global__ void k_unit(double *v, int64_t n, const int64_t *idx, int k, double *vals) {
  // v: [k][n], set v[i][idx[i]] = 1 (assumes zeroed)
  int i = threadIdx.x;
  if (i < k) v[(int64_t)i * n + idx[i]] = 1.0;
}

__global__ void k_gather_sub(const double *X, int64_t n, const int64_t *idx, int k, double *out) {
  int i = threadIdx.x, j = threadIdx.y;
  if (i < k && j < k) out[i * k + j] = X[(int64_t)j * n + idx[i]];
}

int initial_vector(sbci_ctx *ctx, Solver &S) {
  const int64_t n = ctx->ndet;
  double *x = S.v64[X_], *X = S.v64[XX_];
  if (S.o.x0) {
    SBCI_HIP(hipMemcpyAsync(x, S.o.x0, sizeof(double) * n, hipMemcpyHostToDevice, ctx->stream));
    SBCI_TRY(sigma(ctx, x, X, 1, SBCI_F64));
    S.rep.nsigma_f64 += 1;
    const double *xp[1] = {x}, *Xp[1] = {X};
    SBCI_TRY(dots<double>(ctx, n, x, xp, 1, S.red + 40));
    SBCI_TRY(dots<double>(ctx, n, x, Xp, 1, S.red + 41));
    double d[2];
    SBCI_HIP(hipMemcpyAsync(d, S.red + 40, sizeof(double) * 2, hipMemcpyDeviceToHost, ctx->stream));
    SBCI_HIP(hipStreamSynchronize(ctx->stream));
    S.E = d[1] / d[0];
    return SBCI_OK;
  }
  const int k = (int)std::min<int64_t>(S.nroots, n);
  std::vector<int64_t> idx;
  SBCI_TRY(lowest_diagonal(ctx, k, idx));
  double *e = nullptr, *He = nullptr, *sub = nullptr;
  int64_t *didx = nullptr;
  SBCI_HIP(hipMalloc(&e, sizeof(double) * n * k));
  SBCI_HIP(hipMalloc(&He, sizeof(double) * n * k));
  SBCI_HIP(hipMalloc(&sub, sizeof(double) * k * k));
  SBCI_HIP(hipMalloc(&didx, sizeof(int64_t) * k));
  SBCI_HIP(hipMemsetAsync(e, 0, sizeof(double) * n * k, ctx->stream));
  SBCI_HIP(hipMemcpyAsync(didx, idx.data(), sizeof(int64_t) * k, hipMemcpyHostToDevice, ctx->stream));
  k_unit<<<1, 64, 0, ctx->stream>>>(e, n, didx, k, nullptr);
  SBCI_CHECK_LAUNCH();
  SBCI_TRY(sigma(ctx, e, He, k, SBCI_F64));                                  // Eq. S1
  S.rep.nsigma_f64 += k;
  k_gather_sub<<<1, dim3(16, 16), 0, ctx->stream>>>(He, n, didx, k, sub);
  SBCI_CHECK_LAUNCH();
  std::vector<double> Hs((size_t)k * k), w(k), U((size_t)k * k);
  SBCI_HIP(hipMemcpyAsync(Hs.data(), sub, sizeof(double) * k * k, hipMemcpyDeviceToHost, ctx->stream));
  SBCI_HIP(hipStreamSynchronize(ctx->stream));
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < i; ++j) Hs[i * k + j] = Hs[j * k + i] = 0.5 * (Hs[i * k + j] + Hs[j * k + i]);
  jacobi_eigh<16>(k, Hs.data(), w.data(), U.data());
  std::vector<const double *> es(k), Hes(k);
  std::vector<double> cf(k);
  for (int i = 0; i < k; ++i) {
    es[i] = e + (int64_t)i * n;
    Hes[i] = He + (int64_t)i * n;
    cf[i] = U[i * k + 0];
  }
  SBCI_TRY(lincomb<double>(ctx, n, x, es.data(), cf.data(), k, 0.0));      // Eq. S2
  SBCI_TRY(lincomb<double>(ctx, n, X, Hes.data(), cf.data(), k, 0.0));     // Eq. S3
  S.E = w[0];
  SBCI_HIP(hipStreamSynchronize(ctx->stream));
  hipFree(e);
  hipFree(He);
  hipFree(sub);
  hipFree(didx);
  return SBCI_OK;
}

void free_solver(Solver &S) {
  for (int i = 0; i < NV; ++i) {
    hipFree(S.v64[i]);
    hipFree(S.v32[i]);
    S.v64[i] = nullptr;
    S.v32[i] = nullptr;
  }
  for (auto p : S.xc64) hipFree(p);
  for (auto p : S.xc32) hipFree(p);
  S.xc64.clear();
  S.xc32.clear();
  hipFree(S.red);
  S.red = nullptr;
}

int resolve_opts(const sbci_opts *opt, double tol, int nroots, int64_t ndet, sbci_opts &o) {
  if (opt) o = *opt; else sbci_default_opts(&o);
  if (tol > 0) {
    o.eps0 = tol;
    o.r0 = std::sqrt(tol);
  }
  if (nroots < 1 || nroots > 16 || nroots > ndet)
    return set_error(SBCI_EINVAL, "nroots must be in [1, min(16, N_det)]");
  if (!(o.eps0 > 0) || !(o.r0 > 0)) return set_error(SBCI_EINVAL, "eps0 and r0 must be > 0");
  if (o.precision != SBCI_F64 && o.precision != SBCI_F32 && o.precision != SBCI_BF16)
    return set_error(SBCI_EINVAL, "unknown precision");
  if (o.max_cycle < 1 || o.max_steps < 1) return set_error(SBCI_EINVAL, "max_cycle, max_steps >= 1");
  return SBCI_OK;
}

}  // namespace

int solver_begin(sbci_ctx *ctx, int nroots, double tol, const sbci_opts *opt) {
  if (ctx->solver) {
    free_solver(*ctx->solver);
    delete ctx->solver;
    ctx->solver = nullptr;
  }
  Solver *S = new Solver();
  ctx->solver = S;
  SBCI_TRY(resolve_opts(opt, tol, nroots, ctx->ndet, S->o));
  S->nroots = nroots;
  S->n = ctx->ndet;
  S->t0 = now_s();
  ctx->trace.clear();
  SBCI_TRY(alloc_solver(ctx, *S, S->o.precision != SBCI_F64));
  SBCI_TRY(initial_vector(ctx, *S));
  if (S->o.precision != SBCI_F64) {
    SBCI_TRY((convert<float, double>(ctx, S->n, S->v32[X_], S->v64[X_], 1.0)));
    SBCI_TRY((convert<float, double>(ctx, S->n, S->v32[XX_], S->v64[XX_], 1.0)));
    S->phase = S->o.precision;
    return start_root<float>(ctx, *S);
  }
  S->phase = SBCI_F64;
  return start_root<double>(ctx, *S);
}

int solver_step(sbci_ctx *ctx, sbci_step_info *info, int *done) {
  Solver *S = ctx->solver;
  if (!S) return set_error(SBCI_EINVAL, "sbci_step before sbci_begin");
  if (S->done) {
    if (done) *done = 1;
    return SBCI_OK;
  }
  int rc = S->phase == SBCI_F64 ? step_t<double>(ctx, *S, info) : step_t<float>(ctx, *S, info);
  if (done) *done = S->done ? 1 : 0;
  return rc;
}

int solver_finish(sbci_ctx *ctx, double *energies, double *dev_vecs, sbci_report *rep) {
  Solver *S = ctx->solver;
  if (!S) return set_error(SBCI_EINVAL, "sbci_finish before sbci_begin");
  SBCI_HIP(hipStreamSynchronize(ctx->stream));
  const int nc = (int)S->Ec.size();
  for (int i = 0; i < nc && energies; ++i) energies[i] = S->Ec[i];
  if (dev_vecs)
    for (int i = 0; i < nc; ++i)
      SBCI_HIP(hipMemcpyAsync(dev_vecs + (int64_t)i * S->n, S->xc64[i], sizeof(double) * S->n,
                              hipMemcpyDeviceToDevice, ctx->stream));
  SBCI_HIP(hipStreamSynchronize(ctx->stream));
  S->rep.seconds = now_s() - S->t0;
  S->rep.peak_vector_bytes = (int64_t)S->alloc_bytes;
  if (rep) *rep = S->rep;
  if (!S->done) return set_error(SBCI_ENOCONV, "not all roots converged");
  if (S->any_noconv) return set_error(SBCI_ENOCONV, "a root reached max_steps");
  return SBCI_OK;
}

void solver_free(sbci_ctx *ctx) {
  if (ctx->solver) {
    free_solver(*ctx->solver);
    delete ctx->solver;
    ctx->solver = nullptr;
  }
}

// ------------------------------------------------------------ Davidson
namespace {

__global__ void k_precond(int64_t n, const double *__restrict__ r, const double *__restrict__ D,
                          double theta, double fl, double *__restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double den = D[i] - theta;
    if (fabs(den) < fl) den = fl;
    out[i] = r[i] / den;
  }
}

// out = sum_i coef[i] * vs[i], any number of terms (chunks of 16)
int lincomb_n(sbci_ctx *ctx, int64_t n, double *out, const std::vector<const double *> &vs,
              const std::vector<double> &cf, double beta) {
  const int m = (int)vs.size();
  for (int s = 0; s < m || s == 0; s += 16) {
    int cnt = std::min(16, m - s);
    if (cnt <= 0) break;
    SBCI_TRY(lincomb<double>(ctx, n, out, vs.data() + s, cf.data() + s, cnt, s == 0 ? beta : 1.0));
  }
  return SBCI_OK;
}

int dots_n(sbci_ctx *ctx, int64_t n, const double *a, const std::vector<const double *> &vs,
           double *dev_out, std::vector<double> &host) {
  const int m = (int)vs.size();
  for (int s = 0; s < m; s += 16) {
    int cnt = std::min(16, m - s);
    SBCI_TRY(dots<double>(ctx, n, a, vs.data() + s, cnt, dev_out + s));
  }
  host.resize(m);
  SBCI_HIP(hipMemcpyAsync(host.data(), dev_out, sizeof(double) * m, hipMemcpyDeviceToHost, ctx->stream));
  SBCI_HIP(hipStreamSynchronize(ctx->stream));
  return SBCI_OK;
}

}  // namespace

int davidson(sbci_ctx *ctx, int nroots, double tol, const sbci_opts *opt, double *energies,
             double *dev_vecs, sbci_report *rep_out) {
  sbci_opts o;
  SBCI_TRY(resolve_opts(opt, tol, nroots, ctx->ndet, o));
  const int64_t n = ctx->ndet;
  const int maxs = o.max_space > 0 ? o.max_space : 12 + nroots;
  if (maxs < 2 * nroots) return set_error(SBCI_EINVAL, "max_space must be >= 2 * nroots");
  const double t0 = now_s();
  sbci_report rep{};
  struct Buf {
    double *p = nullptr;
    ~Buf() { hipFree(p); }
  } V, W, Xr, Rr, Wr, red;
  SBCI_HIP(hipMalloc(&V.p, sizeof(double) * n * maxs));
  SBCI_HIP(hipMalloc(&W.p, sizeof(double) * n * maxs));
  SBCI_HIP(hipMalloc(&Xr.p, sizeof(double) * n * nroots));
  SBCI_HIP(hipMalloc(&Rr.p, sizeof(double) * n * nroots));
  SBCI_HIP(hipMalloc(&Wr.p, sizeof(double) * n * nroots));
  SBCI_HIP(hipMalloc(&red.p, sizeof(double) * 64));
  rep.peak_vector_bytes = (int64_t)sizeof(double) * n * (2 * maxs + 3 * nroots);
  SBCI_HIP(hipMemsetAsync(V.p, 0, sizeof(double) * n * nroots, ctx->stream));
  std::vector<int64_t> idx;
  SBCI_TRY(lowest_diagonal(ctx, nroots, idx));
  int64_t *didx = nullptr;
  SBCI_HIP(hipMalloc(&didx, sizeof(int64_t) * nroots));
  SBCI_HIP(hipMemcpyAsync(didx, idx.data(), sizeof(int64_t) * nroots, hipMemcpyHostToDevice, ctx->stream));
  k_unit<<<1, 64, 0, ctx->stream>>>(V.p, n, didx, nroots, nullptr);
  SBCI_CHECK_LAUNCH();
  SBCI_HIP(hipStreamSynchronize(ctx->stream));
  hipFree(didx);
  int m = nroots;
  SBCI_TRY(sigma(ctx, V.p, W.p, nroots, SBCI_F64));
  rep.nsigma_f64 += nroots;
  std::vector<double> h((size_t)maxs * maxs, 0.0);
  auto vptr = [&](double *base, int i) { return base + (int64_t)i * n; };
  // fill subspace matrix for columns [c0, m)
  auto fill = [&](int c0) -> int {
    std::vector<const double *> vs(m);
    for (int i = 0; i < m; ++i) vs[i] = vptr(V.p, i);
    std::vector<double> hd;
    for (int j = c0; j < m; ++j) {
      SBCI_TRY(dots_n(ctx, n, vptr(W.p, j), vs, red.p, hd));
      for (int i = 0; i < m; ++i) {
        h[(size_t)i * maxs + j] = hd[i];
        h[(size_t)j * maxs + i] = hd[i];
      }
    }
    for (int i = c0; i < m; ++i)
      for (int j = c0; j < i; ++j) {
        double s = 0.5 * (h[(size_t)i * maxs + j] + h[(size_t)j * maxs + i]);
        h[(size_t)i * maxs + j] = h[(size_t)j * maxs + i] = s;
      }
    return SBCI_OK;
  };
  SBCI_TRY(fill(0));
  std::vector<double> th_old(nroots, INFINITY), th(nroots), tconv(nroots, -1.0);
  std::vector<int> conv(nroots, 0);
  bool all = false;
  int it = 0;
  for (; it < o.max_steps; ++it) {
    std::vector<double> hs((size_t)m * m), w(m), U((size_t)m * m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) hs[i * m + j] = h[(size_t)i * maxs + j];
    jacobi_eigh<32>(m, hs.data(), w.data(), U.data());
    std::vector<const double *> vs(m), ws(m);
    for (int i = 0; i < m; ++i) {
      vs[i] = vptr(V.p, i);
      ws[i] = vptr(W.p, i);
    }
    std::vector<double> rn(nroots);
    for (int k = 0; k < nroots; ++k) {
      th[k] = w[k];
      std::vector<double> cf(m), cr(2 * m);
      for (int i = 0; i < m; ++i) cf[i] = U[i * m + k];
      SBCI_TRY(lincomb_n(ctx, n, vptr(Xr.p, k), vs, cf, 0.0));
      SBCI_TRY(lincomb_n(ctx, n, vptr(Wr.p, k), ws, cf, 0.0));
      std::vector<const double *> rv = {vptr(Wr.p, k), vptr(Xr.p, k)};
      std::vector<double> rc = {1.0, -th[k]};
      SBCI_TRY(lincomb_n(ctx, n, vptr(Rr.p, k), rv, rc, 0.0));
      std::vector<const double *> self = {vptr(Rr.p, k)};
      std::vector<double> d;
      SBCI_TRY(dots_n(ctx, n, vptr(Rr.p, k), self, red.p, d));
      rn[k] = std::sqrt(d[0]);
      conv[k] = std::fabs(th[k] - th_old[k]) < o.eps0 && rn[k] < o.r0;
      if (!conv[k]) tconv[k] = -1.0;
      else if (tconv[k] < 0) tconv[k] = now_s() - t0;
      rep.t_converged[std::min(k, 15)] = tconv[k];
      rep.resid[std::min(k, 15)] = rn[k];
      if (!std::isfinite(th[k]) || !std::isfinite(rn[k]))
        return set_error(SBCI_ENUMERIC, "Davidson: non-finite Ritz value or residual");
    }
    th_old = th;
    rep.nsteps += 1;
    all = std::all_of(conv.begin(), conv.end(), [](int c) { return c != 0; });
    if (all) break;
    int nnew = 0;
    for (int k = 0; k < nroots; ++k) nnew += conv[k] ? 0 : 1;
    if (m + nnew > maxs) {
      // collapse to the current Ritz vectors
      SBCI_HIP(hipMemcpyAsync(V.p, Xr.p, sizeof(double) * n * nroots, hipMemcpyDeviceToDevice, ctx->stream));
      SBCI_HIP(hipMemcpyAsync(W.p, Wr.p, sizeof(double) * n * nroots, hipMemcpyDeviceToDevice, ctx->stream));
      m = nroots;
      std::fill(h.begin(), h.end(), 0.0);
      for (int i = 0; i < m; ++i) h[(size_t)i * maxs + i] = th[i];
      // re-orthonormalisation is implicit: Ritz vectors of an orthonormal basis
    }
    int added = 0;
    for (int k = 0; k < nroots; ++k) {
      if (conv[k]) continue;
      double *tv = vptr(V.p, m + added);
      k_precond<<<1024, 256, 0, ctx->stream>>>(n, vptr(Rr.p, k), ctx->hdiag, th[k], o.precond_floor, tv);
      SBCI_CHECK_LAUNCH();
      for (int pass = 0; pass < 2; ++pass) {
        std::vector<const double *> bs(m + added);
        for (int i = 0; i < m + added; ++i) bs[i] = vptr(V.p, i);
        std::vector<double> d;
        SBCI_TRY(dots_n(ctx, n, tv, bs, red.p, d));
        for (auto &x : d) x = -x;
        SBCI_TRY(lincomb_n(ctx, n, tv, bs, d, 1.0));
      }
      std::vector<const double *> self = {tv};
      std::vector<double> nn;
      SBCI_TRY(dots_n(ctx, n, tv, self, red.p, nn));
      const double nrm = std::sqrt(nn[0]);
      if (!(nrm > std::sqrt(o.lindep))) continue;
      std::vector<const double *> one = {tv};
      std::vector<double> sc = {1.0 / nrm};
      SBCI_TRY(lincomb_n(ctx, n, tv, one, sc, 0.0));
      added += 1;
    }
    if (added == 0) break;
    SBCI_TRY(sigma(ctx, vptr(V.p, m), vptr(W.p, m), added, SBCI_F64));
    rep.nsigma_f64 += added;
    const int c0 = m;
    m += added;
    SBCI_TRY(fill(c0));
  }
  SBCI_HIP(hipStreamSynchronize(ctx->stream));
  for (int k = 0; k < nroots && energies; ++k) energies[k] = th[k];
  if (dev_vecs)
    SBCI_HIP(hipMemcpyAsync(dev_vecs, Xr.p, sizeof(double) * n * nroots, hipMemcpyDeviceToDevice,
                            ctx->stream));
  SBCI_HIP(hipStreamSynchronize(ctx->stream));
  rep.nroots_converged = 0;
  for (int k = 0; k < nroots; ++k) rep.nroots_converged += conv[k];
  rep.seconds = now_s() - t0;
  if (rep_out) *rep_out = rep;
  if (!all) return set_error(SBCI_ENOCONV, "Davidson did not converge");
  return SBCI_OK;
}

}  // namespace sbci
