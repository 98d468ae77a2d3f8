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
  // converged-root storage allocated when a solve begins, taken as roots
  // converge (no allocation inside the step loop)
  std::vector<double *> pool64;
  std::vector<float *> pool32;
  // H x_c of the first Hxc64.size() converged roots (SBCI2 keeps them); where
  // present they replace E_c x_c in the projections of X (Eqs. S5, S78)
  std::vector<double *> Hxc64;
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
  bool stepwise = false;  // begun by solver_begin (SBCI1, one step per call)
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
  if (!ctx->trace_on && !ctx->progress) return;
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
  if (ctx->trace_on) ctx->trace.push_back(r);
  if (ctx->progress) ctx->progress(&r, ctx->progress_user);
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
// energy S.E: the root start of Algorithm 1 (Eqs. S4-S7), then the segment start.
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
    // Eq. S5; roots with a kept image H x_c use it in place of E_c x_c
    const int nimg = std::is_same<T, double>::value ? (int)std::min(S.Hxc64.size(), (size_t)nconv) : 0;
    if (nimg > 0) {
      std::vector<const T *> hp(nimg);
      for (int i = 0; i < nimg; ++i) hp[i] = reinterpret_cast<const T *>(S.Hxc64[i]);
      SBCI_TRY(lincomb<T>(ctx, S.n, X, hp.data(), cx, nimg, 1.0));
    }
    if (nconv > nimg)
      SBCI_TRY(lincomb<T>(ctx, S.n, X, xcp.data() + nimg, cX + nimg, nconv - nimg, 1.0));
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
  if (!(d[0] > 0) || !std::isfinite(d[0]) || !std::isfinite(d[1]))
    return set_error(SBCI_ENUMERIC, "the BF16-phase iterate is not finite at the hand-over");
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
  if (!(d[0] > 0) || !std::isfinite(d[0]) || !std::isfinite(d[1]))
    return set_error(SBCI_ENUMERIC, "the low-precision iterate is not finite at the hand-over");
  S.E = d[1] / d[0];
  S.phase = SBCI_F64;
  int steps = S.steps_root;
  int seg = S.seg;
  SBCI_TRY(start_root<double>(ctx, S));
  S.steps_root = steps;
  S.seg = seg + 1;
  return SBCI_OK;
}

// Hand-over from a low-precision phase to the next rung: BF16 -> FP32,
// FP32 -> FP64.  Both recompute X = H x from x in the new precision.
int next_rung(sbci_ctx *ctx, Solver &S) {
  return S.phase == SBCI_BF16 ? to_f32(ctx, S) : promote(ctx, S);
}

// Finish root alpha in FP64 and prepare the next root's start vector from
// the second Ritz vector of the converging step (Section S1.4).
int finish_root(sbci_ctx *ctx, Solver &S, double xn, bool second_ok) {
  double *xc = nullptr;
  if (!S.pool64.empty()) {
    xc = S.pool64.back();
    S.pool64.pop_back();
  } else {
    SBCI_HIP(hipMalloc(&xc, sizeof(double) * S.n));
    S.alloc_bytes += sizeof(double) * S.n;
  }
  S.xc64.push_back(xc);
  SBCI_TRY((convert<double, double>(ctx, S.n, xc, S.v64[X_], 1.0 / xn)));
  if (S.o.precision != SBCI_F64) {
    float *x32 = nullptr;
    if (!S.pool32.empty()) {
      x32 = S.pool32.back();
      S.pool32.pop_back();
    } else {
      SBCI_HIP(hipMalloc(&x32, sizeof(float) * S.n));
      S.alloc_bytes += sizeof(float) * S.n;
    }
    S.xc32.push_back(x32);
    SBCI_TRY((convert<float, double>(ctx, S.n, x32, xc, 1.0)));
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
  // the Ritz vector goes to the free z slot first; x and X stay intact until
  // its norm is known to be usable
  SBCI_TRY(lincomb<T>(ctx, S.n, S.vec<T>(S.zn), in1, cf, 3, 0.0));
  const T *vp[1] = {S.vec<T>(S.zn)};
  SBCI_TRY(dots<T>(ctx, S.n, S.vec<T>(S.zn), vp, 1, S.red + 40));
  double nxx;
  SBCI_HIP(hipMemcpyAsync(&nxx, S.red + 40, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  SBCI_HIP(hipStreamSynchronize(ctx->stream));
  if (!(nxx > 0) || !std::isfinite(nxx)) {
    if (S.phase != SBCI_F64) return next_rung(ctx, S);
    return set_error(SBCI_ENUMERIC, "SBCI: the Ritz vector of a restart vanished");
  }
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
  bool finite = true;
  for (int i = 0; i < 6; ++i) finite = finite && std::isfinite(N[i]) && std::isfinite(Hm[i]);
  if (!finite) {
    // a low-precision phase hands over (the next rung recomputes X = H x
    // from x); in FP64 there is nothing to fall back to
    if (S.phase != SBCI_F64) return next_rung(ctx, S);
    return set_error(SBCI_ENUMERIC, "non-finite reduction in SBCI step");
  }
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
    if (!(N[0] > 0)) {
      if (S.phase != SBCI_F64) return next_rung(ctx, S);
      return set_error(SBCI_ENUMERIC, "SBCI: x vanished at a rank restart");
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
  if (S.phase != SBCI_F64 && std::fabs(r.k) < S.o.x_th1) {
    // |x_{t+1}| = |k_t| (the Ritz vector has unit norm and x_{t+1} is it
    // divided by its x coefficient), so the update would build x_{t+1} by
    // heavy cancellation.  In a low-precision phase the carried images then
    // no longer match H x to the accuracy the small problem needs (its
    // lowest value can fall below the spectrum and the iterate runs away to
    // overflow), so the step is not taken: the phase hands over from the
    // current x, which is still intact.
    record(ctx, S, r.E[0], NAN, NAN, r.b, r.c, r.k, std::fabs(r.k), 9);
    if (info) *info = ctx->trace.empty() ? sbci_step_info{} : ctx->trace.back();
    return next_rung(ctx, S);
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
  if (promote_now) return next_rung(ctx, S);
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

// Lexicographic (value, index) order of diagonal entries: the order of
// Section S1.1's "lowest diagonal elements" with ties broken by lower index.
__device__ __forceinline__ bool lex_less(double v, int64_t i, double w, int64_t j) {
  return v < w || (v == w && i < j);
}

__device__ __forceinline__ void lex_min_into(double &v, int64_t &i, double w, int64_t j) {
  if (lex_less(w, j, v, i)) {
    v = w;
    i = j;
  }
}

// Per block: the smallest entry of D, in (value, index) order, among those
// above the previous pick (*pv, *pi) (all entries when has_prev = 0).  NaN
// entries are never picked; the sentinel index n means "none".
__global__ __launch_bounds__(256) void k_argmin_above(const double *__restrict__ D, int64_t n,
                                                      const double *__restrict__ pv,
                                                      const int64_t *__restrict__ pi, int has_prev,
                                                      double *__restrict__ bv, int64_t *__restrict__ bi) {
  __shared__ double sv[4];
  __shared__ int64_t si[4];
  const double v0 = has_prev ? *pv : 0.0;
  const int64_t i0 = has_prev ? *pi : -1;
  double best = INFINITY;
  int64_t bidx = n;
  for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double v = D[i];
    if (v == v && (!has_prev || lex_less(v0, i0, v, i))) lex_min_into(best, bidx, v, i);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double w = __shfl_xor(best, o);
    const int64_t j = __shfl_xor(bidx, o);
    lex_min_into(best, bidx, w, j);
  }
  if ((threadIdx.x & 63) == 0) {
    sv[threadIdx.x >> 6] = best;
    si[threadIdx.x >> 6] = bidx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) lex_min_into(best, bidx, sv[w], si[w]);
    bv[blockIdx.x] = best;
    bi[blockIdx.x] = bidx;
  }
}

// The pick: the smallest of nb block results, written to (*ov, *oi).
__global__ __launch_bounds__(64) void k_argmin_final(const double *__restrict__ bv,
                                                     const int64_t *__restrict__ bi, int nb,
                                                     int64_t n, double *__restrict__ ov,
                                                     int64_t *__restrict__ oi) {
  double best = INFINITY;
  int64_t bidx = n;
  for (int b = threadIdx.x; b < nb; b += 64) lex_min_into(best, bidx, bv[b], bi[b]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double w = __shfl_xor(best, o);
    const int64_t j = __shfl_xor(bidx, o);
    lex_min_into(best, bidx, w, j);
  }
  if (threadIdx.x == 0) {
    *ov = best;
    *oi = bidx;
  }
}

// Section S1.1: the nroots lowest diagonal determinants (ties: lower index),
// found on the device: pick j is the smallest entry above pick j - 1 in
// (value, index) order, one read of D per pick, one host copy at the end.
int lowest_diagonal(sbci_ctx *ctx, int k, std::vector<int64_t> &idx) {
  const int64_t n = ctx->ndet;
  const int nb = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + 255) / 256));
  double *buf = nullptr;
  SBCI_HIP(hipMalloc(&buf, sizeof(double) * (2 * (size_t)nb + 2 * (size_t)k)));
  struct Free {
    void *p;
    ~Free() { hipFree(p); }
  } guard{buf};
  double *bv = buf, *ov = buf + nb;
  int64_t *bi = reinterpret_cast<int64_t *>(buf + nb + k);
  int64_t *oi = bi + nb;
  for (int j = 0; j < k; ++j) {
    k_argmin_above<<<nb, 256, 0, ctx->stream>>>(ctx->hdiag, n, j > 0 ? ov + j - 1 : ov,
                                                j > 0 ? oi + j - 1 : oi, j > 0 ? 1 : 0, bv, bi);
    k_argmin_final<<<1, 64, 0, ctx->stream>>>(bv, bi, nb, n, ov + j, oi + j);
    SBCI_CHECK_LAUNCH();
  }
  idx.assign((size_t)k, 0);
  SBCI_HIP(hipMemcpyAsync(idx.data(), oi, sizeof(int64_t) * k, hipMemcpyDeviceToHost, ctx->stream));
  SBCI_HIP(hipStreamSynchronize(ctx->stream));
  for (int j = 0; j < k; ++j)
    if (idx[j] < 0 || idx[j] >= n)
      return set_error(SBCI_ENUMERIC, "start vectors: fewer than nroots finite diagonal entries");
  return SBCI_OK;
}

__global__ void k_unit(double *v, int64_t n, const int64_t *idx, int k, double *vals) {
  // v: [k][n], set v[i][idx[i]] = 1 (assumes zeroed)
  int i = threadIdx.x;
  if (i < k) v[(int64_t)i * n + idx[i]] = 1.0;
}

__global__ void k_sparse_set(double *v, const int64_t *idx, const double *val, int k) {
  const int i = threadIdx.x;
  if (i < k) v[idx[i]] = val[i];
}

__global__ void k_gather_rows(const double *v, const int64_t *idx, int k, double *out) {
  const int i = threadIdx.x;
  if (i < k) out[i] = v[idx[i]];
}

// The k x k block of H on the k lowest diagonal determinants (Sections S1.1,
// S2.2) and its eigenpairs: column j is gathered from sigma of the unit
// vector e_j, one column at a time, so only the two scratch vectors e, He
// ([n] each) are needed.  w ascending; U[i * k + a] = coefficient of
// e_{idx[i]} in eigenvector a.
int start_block(sbci_ctx *ctx, int k, double *e, double *He, std::vector<int64_t> &idx,
                std::vector<double> &w, std::vector<double> &U, int64_t &nsig) {
  const int64_t n = ctx->ndet;
  SBCI_TRY(lowest_diagonal(ctx, k, idx));
  int64_t *didx = nullptr;
  double *dval = nullptr;
  SBCI_HIP(hipMalloc(&didx, sizeof(int64_t) * k));
  SBCI_HIP(hipMalloc(&dval, sizeof(double) * 2 * k));
  struct Free {
    void *a, *b;
    ~Free() { hipFree(a); hipFree(b); }
  } guard{didx, dval};
  SBCI_HIP(hipMemcpyAsync(didx, idx.data(), sizeof(int64_t) * k, hipMemcpyHostToDevice, ctx->stream));
  const double one = 1.0;
  SBCI_HIP(hipMemcpyAsync(dval, &one, sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  std::vector<double> Hs((size_t)k * k), col(k);
  for (int j = 0; j < k; ++j) {
    SBCI_HIP(hipMemsetAsync(e, 0, sizeof(double) * n, ctx->stream));
    k_sparse_set<<<1, 64, 0, ctx->stream>>>(e, didx + j, dval, 1);
    SBCI_CHECK_LAUNCH();
    SBCI_TRY(sigma(ctx, e, He, 1, SBCI_F64));                                // Eqs. S1 / S74
    k_gather_rows<<<1, 64, 0, ctx->stream>>>(He, didx, k, dval + k);
    SBCI_CHECK_LAUNCH();
    SBCI_HIP(hipMemcpyAsync(col.data(), dval + k, sizeof(double) * k, hipMemcpyDeviceToHost,
                            ctx->stream));
    SBCI_HIP(hipStreamSynchronize(ctx->stream));
    for (int i = 0; i < k; ++i) Hs[(size_t)i * k + j] = col[i];
  }
  nsig += k;
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < i; ++j) Hs[i * k + j] = Hs[j * k + i] = 0.5 * (Hs[i * k + j] + Hs[j * k + i]);
  w.assign(k, 0.0);
  U.assign((size_t)k * k, 0.0);
  jacobi_eigh<16>(k, Hs.data(), w.data(), U.data());
  return SBCI_OK;
}

// Start vector a of the block (Eqs. S2 / S75): x = sum_i U[i][a] e_{idx[i]}
// (k non-zeros) and its image X = H x by one sigma, which equals the
// combination of the unit vectors' images (Eqs. S3 / S76) without keeping
// those images.
int start_vector(sbci_ctx *ctx, int k, const std::vector<int64_t> &idx,
                 const std::vector<double> &U, int a, double *x, double *X, int64_t &nsig) {
  const int64_t n = ctx->ndet;
  int64_t *didx = nullptr;
  double *dval = nullptr;
  SBCI_HIP(hipMalloc(&didx, sizeof(int64_t) * k));
  SBCI_HIP(hipMalloc(&dval, sizeof(double) * k));
  struct Free {
    void *a, *b;
    ~Free() { hipFree(a); hipFree(b); }
  } guard{didx, dval};
  std::vector<double> v(k);
  for (int i = 0; i < k; ++i) v[i] = U[(size_t)i * k + a];
  SBCI_HIP(hipMemcpyAsync(didx, idx.data(), sizeof(int64_t) * k, hipMemcpyHostToDevice, ctx->stream));
  SBCI_HIP(hipMemcpyAsync(dval, v.data(), sizeof(double) * k, hipMemcpyHostToDevice, ctx->stream));
  SBCI_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, ctx->stream));
  k_sparse_set<<<1, 64, 0, ctx->stream>>>(x, didx, dval, k);
  SBCI_CHECK_LAUNCH();
  SBCI_TRY(sigma(ctx, x, X, 1, SBCI_F64));
  nsig += 1;
  SBCI_HIP(hipStreamSynchronize(ctx->stream));  // host staging above must outlive the copies
  return SBCI_OK;
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
  // a resumed solve starts root alpha from the start block's vector alpha
  // (the lower ones are projected off by the root start)
  const int a = (int)S.Ec.size();
  std::vector<int64_t> idx;
  std::vector<double> w, U;
  // the solver's y and Y slots are free until the first step
  SBCI_TRY(start_block(ctx, k, S.v64[Y_], S.v64[YY_], idx, w, U, S.rep.nsigma_f64));
  SBCI_HIP(hipMemsetAsync(S.v64[Y_], 0, sizeof(double) * n, ctx->stream));
  SBCI_HIP(hipMemsetAsync(S.v64[YY_], 0, sizeof(double) * n, ctx->stream));
  SBCI_TRY(start_vector(ctx, k, idx, U, a, x, X, S.rep.nsigma_f64));         // Eqs. S2-S3
  S.E = w[a];
  return SBCI_OK;
}

// Resume: the caller's nconv0 converged roots become x_c (orthonormalised in
// the given order by Gram-Schmidt, in FP64) with energies E_c (given, or the
// Rayleigh quotients x_c^T H x_c), exactly as if this solve had converged
// them; the state the solver deflates against is nothing more than {x_c, E_c}.
int resume_roots(sbci_ctx *ctx, Solver &S) {
  const int64_t n = S.n;
  double *X = S.v64[XX_];
  for (int i = 0; i < S.o.nconv0; ++i) {
    double *xc = S.pool64.back();
    S.pool64.pop_back();
    SBCI_HIP(hipMemcpyAsync(xc, S.o.xc0 + (int64_t)i * n, sizeof(double) * n, hipMemcpyHostToDevice,
                            ctx->stream));
    const double *self[1] = {xc};
    double d[16];
    SBCI_TRY(dots<double>(ctx, n, xc, self, 1, S.red + 40));
    SBCI_HIP(hipMemcpyAsync(d, S.red + 40, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    SBCI_HIP(hipStreamSynchronize(ctx->stream));
    const double n0 = d[0];
    if (!(n0 > 0) || !std::isfinite(n0)) {
      hipFree(xc);
      return set_error(SBCI_EINVAL, "resume: a converged vector is zero or not finite");
    }
    S.xc64.push_back(xc);
    if (i > 0) {
      std::vector<const double *> xcp(S.xc64.begin(), S.xc64.end() - 1);
      double cf[16];
      for (int pass = 0; pass < 2; ++pass) {   // two passes: orthogonal to rounding
        SBCI_TRY(dots<double>(ctx, n, xc, xcp.data(), i, S.red + 40));
        SBCI_HIP(hipMemcpyAsync(d, S.red + 40, sizeof(double) * i, hipMemcpyDeviceToHost, ctx->stream));
        SBCI_HIP(hipStreamSynchronize(ctx->stream));
        for (int j = 0; j < i; ++j) cf[j] = -d[j];
        SBCI_TRY(lincomb<double>(ctx, n, xc, xcp.data(), cf, i, 1.0));
      }
    }
    SBCI_TRY(dots<double>(ctx, n, xc, self, 1, S.red + 40));
    SBCI_HIP(hipMemcpyAsync(d, S.red + 40, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    SBCI_HIP(hipStreamSynchronize(ctx->stream));
    if (!(d[0] > S.o.lindep * n0))
      return set_error(SBCI_EINVAL, "resume: the converged vectors are linearly dependent");
    SBCI_TRY((convert<double, double>(ctx, n, xc, xc, 1.0 / std::sqrt(d[0]))));
    double E;
    if (S.o.ec0) {
      E = S.o.ec0[i];
      if (!std::isfinite(E)) return set_error(SBCI_EINVAL, "resume: a converged energy is not finite");
    } else {
      SBCI_TRY(sigma(ctx, xc, X, 1, SBCI_F64));
      S.rep.nsigma_f64 += 1;
      const double *Xp[1] = {X};
      SBCI_TRY(dots<double>(ctx, n, xc, Xp, 1, S.red + 40));
      SBCI_HIP(hipMemcpyAsync(&E, S.red + 40, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
      SBCI_HIP(hipStreamSynchronize(ctx->stream));
    }
    if (S.o.precision != SBCI_F64) {
      float *x32 = S.pool32.back();
      S.pool32.pop_back();
      S.xc32.push_back(x32);
      SBCI_TRY((convert<float, double>(ctx, n, x32, xc, 1.0)));
    }
    S.Ec.push_back(E);
  }
  S.alpha = S.o.nconv0;
  S.rep.nroots_converged = S.o.nconv0;
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
  for (auto p : S.Hxc64) hipFree(p);
  for (auto p : S.pool64) hipFree(p);
  for (auto p : S.pool32) hipFree(p);
  S.xc64.clear();
  S.xc32.clear();
  S.Hxc64.clear();
  S.pool64.clear();
  S.pool32.clear();
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
  if (o.s78_printed != 0 && o.s78_printed != 1) return set_error(SBCI_EINVAL, "s78_printed must be 0 or 1");
  if (o.nconv0 < 0 || o.nconv0 >= nroots)
    return set_error(SBCI_EINVAL, "nconv0 must be in [0, nroots)");
  if (o.nconv0 > 0 && !o.xc0) return set_error(SBCI_EINVAL, "nconv0 > 0 needs xc0");
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
  for (int i = 0; i < nroots; ++i) {
    double *p = nullptr;
    SBCI_HIP(hipMalloc(&p, sizeof(double) * S->n));
    S->pool64.push_back(p);
    S->alloc_bytes += sizeof(double) * S->n;
    if (S->o.precision != SBCI_F64) {
      float *q = nullptr;
      SBCI_HIP(hipMalloc(&q, sizeof(float) * S->n));
      S->pool32.push_back(q);
      S->alloc_bytes += sizeof(float) * S->n;
    }
  }
  S->stepwise = true;
  SBCI_TRY(resume_roots(ctx, *S));
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

// The current iterate x of the root being solved, in FP64.  Between steps
// it is held unnormalised (the pending scale is positive), so its direction
// is exact; with {x_c, E_c} it is the whole state at a step boundary.
int solver_iterate(sbci_ctx *ctx, double *dev_x) {
  Solver *S = ctx->solver;
  if (!S || !S->stepwise) return set_error(SBCI_EINVAL, "sbci_iterate needs an SBCI1 solve begun by sbci_begin or sbci_solve");
  if (S->done) return set_error(SBCI_EINVAL, "sbci_iterate: every root has converged");
  if (S->phase == SBCI_F64)
    SBCI_TRY((convert<double, double>(ctx, S->n, dev_x, S->v64[X_], 1.0)));
  else
    SBCI_TRY((convert<double, float>(ctx, S->n, dev_x, S->v32[X_], 1.0)));
  SBCI_HIP(hipStreamSynchronize(ctx->stream));
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
  if (o.nconv0 != 0) return set_error(SBCI_EINVAL, "sbci_davidson does not resume (nconv0 must be 0)");
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
    all = std::all_of(conv.begin(), conv.end(), [](int c) { return c != 0; });
    if (ctx->progress) {
      int k0 = 0;
      while (k0 < nroots - 1 && conv[k0]) ++k0;
      sbci_step_info r{};
      r.root = k0;
      r.t = it;
      r.precision = SBCI_F64;
      r.E = th[k0];
      r.dE = std::fabs(th[k0] - th_old[k0]);
      r.dz = rn[k0];
      r.b = r.c = r.k = r.xnorm = NAN;
      r.seconds = now_s() - t0;
      r.reason = all ? 1 : 0;
      ctx->progress(&r, ctx->progress_user);
    }
    th_old = th;
    rep.nsteps += 1;
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

// ------------------------------------------------------------ SBCI2
// SBCI2 (Algorithm 2; Sections S2.1-S2.5).  The states of a pair
// (alpha, alpha + 1) advance together: per step both preconditioned,
// deflated residuals get their sigma images in one two-vector sigma call;
// the overlap and H matrices of the basis (x^a, x^a+1, [y^a, y^a+1,]
// z^a, z^a+1) come from FP64 dot passes; the host orthonormalises the basis
// canonically, solves the small eigenproblem and derives A, B, C (Eqs. S93,
// S112-S121); linear-combination passes update y, Y, x, X (Eqs. S94-S97,
// S122-S125); one fused pass per state forms the next residual.  State alpha
// is accepted on Eq. S127; the pair restarts on S130a-c or after max_cycle
// (10) steps.  The highest state is finished by SBCI1 (Fig. 1B).
namespace sbci {
namespace {

struct Pair {
  double *x[2] = {}, *X[2] = {}, *y[2] = {}, *Y[2] = {};
  double *z = nullptr, *Z = nullptr;  // [2][n] each (one sigma call, nvec = 2)
  double *s[2] = {}, *S[2] = {};      // scratch: Ritz vectors of a restart and their images
  float *z32 = nullptr, *Z32 = nullptr;  // [2][n]: the low-precision phases' sigma operands
  double *dev = nullptr;              // reduction results
  // the k x k block of Eq. S74 on the lowest diagonal determinants: its
  // eigenvectors U give the start vectors of Eq. S75, rebuilt when needed
  int k = 0;
  std::vector<int64_t> idx;
  std::vector<double> U, w;
  size_t bytes = 0;
};

void free_pair(Pair &P) {
  for (int i = 0; i < 2; ++i) {
    hipFree(P.x[i]);
    hipFree(P.X[i]);
    hipFree(P.y[i]);
    hipFree(P.Y[i]);
    hipFree(P.s[i]);
    hipFree(P.S[i]);
  }
  hipFree(P.z);
  hipFree(P.Z);
  hipFree(P.z32);
  hipFree(P.Z32);
  hipFree(P.dev);
}

int dmalloc(Pair &P, double **p, size_t count) {
  SBCI_HIP(hipMalloc(p, sizeof(double) * count));
  P.bytes += sizeof(double) * count;
  return SBCI_OK;
}

// host copies of dots a . b_j (j < nb)
int dots_h(sbci_ctx *ctx, Pair &P, int64_t n, const double *a, const double *const *bs, int nb,
           double *host) {
  SBCI_TRY(dots<double>(ctx, n, a, bs, nb, P.dev));
  SBCI_HIP(hipMemcpyAsync(host, P.dev, sizeof(double) * nb, hipMemcpyDeviceToHost, ctx->stream));
  SBCI_HIP(hipStreamSynchronize(ctx->stream));
  return SBCI_OK;
}

// Z = sigma(z) for the pair's two residuals in the phase's precision: the
// low-precision phases convert z to FP32, run the FP32 or BF16-MFMA sigma
// and widen the result (the vectors and every reduction stay FP64).
int pair_sigma(sbci_ctx *ctx, Solver &S, Pair &P, int phase, const double *z, double *Z) {
  const int64_t n2 = 2 * S.n;
  if (phase == SBCI_F64) {
    SBCI_TRY(sigma(ctx, z, Z, 2, SBCI_F64));
    S.rep.nsigma_f64 += 2;
    return SBCI_OK;
  }
  SBCI_TRY((convert<float, double>(ctx, n2, P.z32, z, 1.0)));
  SBCI_TRY(sigma(ctx, P.z32, P.Z32, 2, phase));
  SBCI_TRY((convert<double, float>(ctx, n2, Z, P.Z32, 1.0)));
  S.rep.nsigma_low += 2;
  if (phase == SBCI_BF16) S.rep.nsigma_bf16 += 2;
  return SBCI_OK;
}

// Hand-over of the pair to the next precision (the ladder of the precision
// form): x normalised, X = sigma(x) recomputed in the new precision (the
// carried X holds the previous sigma's error), E the Rayleigh quotients.
int pair_rebase(sbci_ctx *ctx, Solver &S, Pair &P, int phase, double *E) {
  const int64_t n = S.n;
  for (int i = 0; i < 2; ++i) {
    const double *bs[1] = {P.x[i]};
    double d;
    SBCI_TRY(dots_h(ctx, P, n, P.x[i], bs, 1, &d));
    if (!(d > 0) || !std::isfinite(d)) return set_error(SBCI_ENUMERIC, "SBCI2: vanishing vector");
    SBCI_TRY((convert<double, double>(ctx, n, P.z + i * n, P.x[i], 1.0 / std::sqrt(d))));
    SBCI_TRY((convert<double, double>(ctx, n, P.x[i], P.z + i * n, 1.0)));
  }
  SBCI_TRY(pair_sigma(ctx, S, P, phase, P.z, P.Z));
  for (int i = 0; i < 2; ++i) {
    SBCI_TRY((convert<double, double>(ctx, n, P.X[i], P.Z + i * n, 1.0)));
    const double *bs[1] = {P.X[i]};
    SBCI_TRY(dots_h(ctx, P, n, P.x[i], bs, 1, &E[i]));
  }
  return SBCI_OK;
}

// Section S2.2 / Eq. S74: the k lowest diagonal determinants and H in their
// span diagonalised (its eigenvectors give the start vectors of Eq. S75).
int pair_start_vectors(sbci_ctx *ctx, Solver &S, Pair &P, int k) {
  // scratch: the pair's y slots (unused until the first step)
  P.k = k;
  SBCI_TRY(start_block(ctx, k, P.y[0], P.y[1], P.idx, P.w, P.U, S.rep.nsigma_f64));   // Eq. S74
  for (int i = 0; i < 2; ++i)
    SBCI_HIP(hipMemsetAsync(P.y[i], 0, sizeof(double) * ctx->ndet, ctx->stream));
  return SBCI_OK;
}

// v <- v - sum_j x_c^j (x_c^j . v), V <- V - sum_j (H x_c^j) (x_c^j . v)
// (Eqs. S77-S78).  Eq. S78 writes E_c^j x_c^j for H x_c^j, exact only for an
// exact eigenvector; an accepted x_c^j keeps a residual, and E_c x_c would
// leave it in V for the rest of the run, shifting the later Ritz energies at
// first order.  The image carried to acceptance is H x_c^j up to rounding.
// With opts.s78_printed the images are projected with E_c^j x_c^j as printed.
int project_off(sbci_ctx *ctx, Solver &S, Pair &P, double *v, double *V) {
  const int nc = (int)S.Ec.size();
  if (nc == 0) return SBCI_OK;
  const bool printed = S.o.s78_printed != 0;
  if (!printed && (int)S.Hxc64.size() != nc)
    return set_error(SBCI_ENUMERIC, "SBCI2: internal: a converged root has no image");
  std::vector<const double *> xcp(S.xc64.begin(), S.xc64.end());
  double d[16];
  SBCI_TRY(dots_h(ctx, P, S.n, v, xcp.data(), nc, d));
  double cx[16], cE[16];
  for (int j = 0; j < nc; ++j) {
    cx[j] = -d[j];
    cE[j] = -S.Ec[j] * d[j];
  }
  SBCI_TRY(lincomb<double>(ctx, S.n, v, xcp.data(), cx, nc, 1.0));
  if (printed) {
    SBCI_TRY(lincomb<double>(ctx, S.n, V, xcp.data(), cE, nc, 1.0));
  } else {
    std::vector<const double *> hcp(S.Hxc64.begin(), S.Hxc64.end());
    SBCI_TRY(lincomb<double>(ctx, S.n, V, hcp.data(), cx, nc, 1.0));
  }
  return SBCI_OK;
}

// Canonical orthogonalisation and Rayleigh-Ritz in an m-vector basis
// (Eqs. S83-S87, S103-S107): returns false if fewer than two basis vectors
// survive the 1e-14 overlap cut.  w ascending, Vp[k * r + i] = coefficient
// of basis vector k in Ritz vector i (r kept vectors).
bool canonical_ritz(int m, const double *Sm, const double *Hm, double lindep, double *w, double *Vp,
                    int &r) {
  double s[6], U[36];
  jacobi_eigh<6>(m, Sm, s, U);
  int keep[6];
  r = 0;
  for (int i = 0; i < m; ++i)
    if (s[i] > lindep) keep[r++] = i;
  if (r < 2) return false;
  double Pm[36];  // m x r
  for (int k = 0; k < m; ++k)
    for (int j = 0; j < r; ++j) Pm[k * r + j] = U[k * m + keep[j]] / std::sqrt(s[keep[j]]);
  double Hp[36];
  for (int a = 0; a < r; ++a)
    for (int b = 0; b < r; ++b) {
      double acc = 0;
      for (int k = 0; k < m; ++k)
        for (int l = 0; l < m; ++l) acc += Pm[k * r + a] * Hm[k * m + l] * Pm[l * r + b];
      Hp[a * r + b] = acc;
    }
  for (int a = 0; a < r; ++a)
    for (int b = 0; b < a; ++b) Hp[a * r + b] = Hp[b * r + a] = 0.5 * (Hp[a * r + b] + Hp[b * r + a]);
  double V[36];
  jacobi_eigh<6>(r, Hp, w, V);
  for (int k = 0; k < m; ++k)
    for (int i = 0; i < r; ++i) {
      double acc = 0;
      for (int j = 0; j < r; ++j) acc += Pm[k * r + j] * V[j * r + i];
      Vp[k * r + i] = acc;  // V' = P V
    }
  return true;
}

struct PairCoef {
  double k[2], A01, A10, B[2][2], C[2][2];
};

// Eqs. S92-S93 (first step; basis x^a, x^a+1, z^a, z^a+1)
bool pair_coef_first(const double *Vp, int r, double lindep, PairCoef &c) {
  auto V = [&](int k, int i) { return Vp[k * r + i]; };
  const double d0 = V(0, 0), d1 = V(1, 1);
  if (std::fabs(d0) < lindep || std::fabs(d1) < lindep) return false;
  c.k[0] = 1.0 / d0;
  c.k[1] = 1.0 / d1;
  c.A01 = V(1, 0) / d0;
  c.A10 = V(0, 1) / d1;
  c.B[0][0] = c.B[1][1] = 1.0;
  c.B[0][1] = c.B[1][0] = 0.0;
  c.C[0][0] = -V(2, 0) / d0;
  c.C[0][1] = -V(3, 0) / d0;
  c.C[1][0] = -V(2, 1) / d1;
  c.C[1][1] = -V(3, 1) / d1;
  return true;
}

// Eqs. S112-S121 (later steps; basis x^a, x^a+1, y^a, y^a+1, z^a, z^a+1)
bool pair_coef_next(const double *Vp, int r, double lindep, PairCoef &c) {
  auto V = [&](int k, int i) { return Vp[k * r + i]; };
  if (std::fabs(V(2, 0)) < lindep || std::fabs(V(3, 1)) < lindep) return false;
  c.A01 = V(1, 0) / V(2, 0);                                   // S116
  c.A10 = V(0, 1) / V(3, 1);
  const double den0 = V(0, 0) - V(3, 0) * c.A10, den1 = V(1, 1) - V(2, 1) * c.A01;  // S117
  if (std::fabs(den0) < lindep || std::fabs(den1) < lindep) return false;
  c.k[0] = 1.0 / den0;
  c.k[1] = 1.0 / den1;
  c.B[0][0] = c.k[0] * V(2, 0);                                // S112
  c.B[0][1] = c.k[0] * V(3, 0);
  c.B[1][0] = c.k[1] * V(2, 1);
  c.B[1][1] = c.k[1] * V(3, 1);
  const double m00 = V(2, 0), m01 = V(3, 0), m10 = V(2, 1), m11 = V(3, 1);
  const double det = m00 * m11 - m01 * m10;
  const double mx = std::max(std::max(std::fabs(m00), std::fabs(m01)), std::max(std::fabs(m10), std::fabs(m11)));
  if (!(std::fabs(det) > lindep * std::max(mx * mx, 1e-300))) return false;
  const double r00 = V(4, 0), r01 = V(5, 0), r10 = V(4, 1), r11 = V(5, 1);
  // C = -M^-1 R  (Eq. S121)
  c.C[0][0] = -(m11 * r00 - m01 * r10) / det;
  c.C[0][1] = -(m11 * r01 - m01 * r11) / det;
  c.C[1][0] = -(-m10 * r00 + m00 * r10) / det;
  c.C[1][1] = -(-m10 * r01 + m00 * r11) / det;
  return true;
}

void record_pair(sbci_ctx *ctx, Solver &S, int seg, int t, double E, double dE, double dz,
                 const PairCoef *c, double xn, int reason) {
  if (!ctx->trace_on && !ctx->progress) return;
  sbci_step_info r{};
  r.root = S.alpha;
  r.segment = seg;
  r.t = t;
  r.precision = S.phase;
  r.E = E;
  r.dE = dE;
  r.dz = dz;
  r.b = c ? c->B[0][0] : NAN;
  r.c = c ? c->C[0][0] : NAN;
  r.k = c ? c->k[0] : NAN;
  r.xnorm = xn;
  r.seconds = now_s() - S.t0;
  r.reason = reason;
  if (ctx->trace_on) ctx->trace.push_back(r);
  if (ctx->progress) ctx->progress(&r, ctx->progress_user);
}

// residuals of both states into the z pair (deflated), |z'|^2 into dz2
int pair_residuals(sbci_ctx *ctx, Solver &S, Pair &P, const double *E, const double *inv,
                   double E0, double *dz2) {
  const int nc = (int)S.Ec.size();
  std::vector<const double *> xcp(S.xc64.begin(), S.xc64.end());
  for (int i = 0; i < 2; ++i) {
    double *zi = P.z + (int64_t)i * S.n;
    SBCI_TRY(resid<double>(ctx, S.n, P.x[i], P.X[i], ctx->hdiag, E[i], inv[i], E0, S.o.precond_floor,
                           xcp.data(), nc, zi, P.dev + 16 * i));                  // S98/S100, S101
    if (nc > 0)
      SBCI_TRY(deflate<double>(ctx, S.n, zi, P.x[i], P.x[i], xcp.data(), nc, P.dev + 16 * i + 1,
                               P.dev + 40 + 4 * i));
  }
  double h[32];
  SBCI_HIP(hipMemcpyAsync(h, P.dev, sizeof(double) * 32, hipMemcpyDeviceToHost, ctx->stream));
  SBCI_HIP(hipStreamSynchronize(ctx->stream));
  dz2[0] = h[0];
  dz2[1] = h[16];
  return SBCI_OK;
}

int scale2(sbci_ctx *ctx, Solver &S, double *v, double s) {
  return convert<double, double>(ctx, S.n, v, v, s);
}

}  // namespace

int sbci2_solve(sbci_ctx *ctx, int nroots, double tol, const sbci_opts *opt, double *energies,
                double *dev_vecs, sbci_report *rep_out) {
  solver_free(ctx);
  Solver *Sp = new Solver();
  ctx->solver = Sp;
  Solver &S = *Sp;
  SBCI_TRY(resolve_opts(opt, tol, nroots, ctx->ndet, S.o));
  if (S.o.nconv0 != 0) return set_error(SBCI_EINVAL, "sbci_solve2 does not resume (nconv0 must be 0)");
  const int first_phase = S.o.precision;  // each pair starts here and ends in FP64
  S.nroots = nroots;
  S.n = ctx->ndet;
  S.t0 = now_s();
  S.phase = SBCI_F64;
  ctx->trace.clear();
  SBCI_TRY(alloc_solver(ctx, S, first_phase != SBCI_F64));
  const int64_t n = S.n;
  const int max_cycle2 = S.o.max_cycle2 > 0 ? S.o.max_cycle2 : 10;
  Pair P;
  struct Guard {
    Pair &p;
    ~Guard() { free_pair(p); }
  } guard{P};
  double *xa = nullptr, *Xa = nullptr;  // start of the highest state (SBCI1)
  if (nroots >= 2) {
    for (int i = 0; i < 2; ++i) {
      SBCI_TRY(dmalloc(P, &P.x[i], n));
      SBCI_TRY(dmalloc(P, &P.X[i], n));
      SBCI_TRY(dmalloc(P, &P.y[i], n));
      SBCI_TRY(dmalloc(P, &P.Y[i], n));
      SBCI_TRY(dmalloc(P, &P.s[i], n));
      SBCI_TRY(dmalloc(P, &P.S[i], n));
    }
    SBCI_TRY(dmalloc(P, &P.z, 2 * n));
    SBCI_TRY(dmalloc(P, &P.Z, 2 * n));
    if (first_phase != SBCI_F64) {
      SBCI_HIP(hipMalloc(&P.z32, sizeof(float) * 2 * n));
      SBCI_HIP(hipMalloc(&P.Z32, sizeof(float) * 2 * n));
      P.bytes += sizeof(float) * 4 * n;
    }
    SBCI_TRY(dmalloc(P, &P.dev, 128));
    SBCI_TRY(pair_start_vectors(ctx, S, P, nroots));
    // pair (0, 1) from Eq. S75
    for (int i = 0; i < 2; ++i)
      SBCI_TRY(start_vector(ctx, P.k, P.idx, P.U, i, P.x[i], P.X[i], S.rep.nsigma_f64));
  }
  for (int alpha = 0; alpha + 1 < nroots; ++alpha) {
    S.alpha = alpha;
    // the pair start of Algorithm 2 (Eqs. S77-S80)
    double E[2];
    for (int i = 0; i < 2; ++i) {
      SBCI_TRY(project_off(ctx, S, P, P.x[i], P.X[i]));
      const double *bs[2] = {P.x[i], P.X[i]};
      double d[2];
      SBCI_TRY(dots_h(ctx, P, n, P.x[i], bs, 2, d));
      if (!(d[0] > 0) || !std::isfinite(d[0]))
        return set_error(SBCI_ENUMERIC, "SBCI2: start vector vanished after projection");
      SBCI_TRY(scale2(ctx, S, P.x[i], 1.0 / std::sqrt(d[0])));
      SBCI_TRY(scale2(ctx, S, P.X[i], 1.0 / std::sqrt(d[0])));
      E[i] = d[1] / d[0];
    }
    int seg = 0, steps = 0;
    bool conv = false, capped = false;
    double inv[2] = {1.0, 1.0}, dz2[2];
    double xn[2] = {1.0, 1.0};
    int phase = first_phase;
    int stall = 0;
    double bestE = E[0];
    S.phase = phase;  // recorded with each pair step
    // low-precision phases: state alpha hands over (instead of converging)
    // at the phase's thresholds or after mix_stall steps without a decrease
    auto hand_over = [&](double Ea, double dEa, double dza) {
      if (phase == SBCI_F64) return false;
      if (Ea < bestE - 1e-15 * std::fabs(bestE)) {
        bestE = Ea;
        stall = 0;
      } else {
        stall += 1;
      }
      const bool bf = phase == SBCI_BF16;
      const double e0 = bf ? S.o.bf16_eps0 : S.o.mix_eps0, r0 = bf ? S.o.bf16_r0 : S.o.mix_r0;
      return (dEa < e0 && dza < r0) || stall >= S.o.mix_stall || steps >= S.o.max_steps;
    };
    auto next_phase = [&]() {
      phase = phase == SBCI_BF16 ? SBCI_F32 : SBCI_F64;
      S.phase = phase;
      stall = 0;
      const int rc = pair_rebase(ctx, S, P, phase, E);
      bestE = E[0];
      return rc;
    };
    while (!conv && !capped) {
      // segment start: y = Y = 0, B = I, residuals of x
      int t = 0;
      SBCI_TRY(pair_residuals(ctx, S, P, E, inv, alpha == 0 ? E[0] : S.Ec[0], dz2));
      while (true) {
        SBCI_TRY(pair_sigma(ctx, S, P, phase, P.z, P.Z));                      // S82 / S102
        S.rep.nsteps += 1;
        steps += 1;
        const double *z[2] = {P.z, P.z + n};
        const double *Z[2] = {P.Z, P.Z + n};
        const double *basis[6], *img[6];
        int m = 0;
        for (int i = 0; i < 2; ++i, ++m) {
          basis[m] = P.x[i];
          img[m] = P.X[i];
        }
        if (t > 0)
          for (int i = 0; i < 2; ++i, ++m) {
            basis[m] = P.y[i];
            img[m] = P.Y[i];
          }
        for (int i = 0; i < 2; ++i, ++m) {
          basis[m] = z[i];
          img[m] = Z[i];
        }
        double Sm[36], Hm[36];
        {
          double g[42];
          const int np = m * (m + 1) / 2;
          SBCI_TRY(gram(ctx, n, basis, img, m, P.dev));
          SBCI_HIP(hipMemcpyAsync(g, P.dev, sizeof(double) * 2 * np, hipMemcpyDeviceToHost,
                                  ctx->stream));
          SBCI_HIP(hipStreamSynchronize(ctx->stream));
          int q = 0;
          for (int i = 0; i < m; ++i)
            for (int j = i; j < m; ++j, ++q) {
              Sm[i * m + j] = Sm[j * m + i] = g[q];
              Hm[i * m + j] = Hm[j * m + i] = g[np + q];  // H on the right vector
            }
        }
        for (int i = 0; i < m * m; ++i)
          if (!std::isfinite(Sm[i]) || !std::isfinite(Hm[i]))
            return set_error(SBCI_ENUMERIC, "SBCI2: non-finite reduction");
        double w[6], Vp[36];
        int r = 0;
        PairCoef cf{};
        const bool rok = canonical_ritz(m, Sm, Hm, S.o.lindep, w, Vp, r);
        const bool cok = rok && (t == 0 ? pair_coef_first(Vp, r, S.o.lindep, cf)
                                        : pair_coef_next(Vp, r, S.o.lindep, cf));
        if (!cok) {
          // restart the pair from its two lowest Ritz vectors
          if (rok) {
            for (int i = 0; i < 2; ++i) {
              double c1[6];
              for (int k = 0; k < m; ++k) c1[k] = Vp[k * r + i];
              SBCI_TRY(lincomb<double>(ctx, n, P.s[i], basis, c1, m, 0.0));
              SBCI_TRY(lincomb<double>(ctx, n, P.S[i], img, c1, m, 0.0));
            }
            for (int i = 0; i < 2; ++i) {
              std::swap(P.x[i], P.s[i]);
              std::swap(P.X[i], P.S[i]);
              E[i] = w[i];
            }
          }
          for (int i = 0; i < 2; ++i) {
            const double *bs[2] = {P.x[i], P.X[i]};
            double d[2];
            SBCI_TRY(dots_h(ctx, P, n, P.x[i], bs, 2, d));
            SBCI_TRY(scale2(ctx, S, P.x[i], 1.0 / std::sqrt(d[0])));
            SBCI_TRY(scale2(ctx, S, P.X[i], 1.0 / std::sqrt(d[0])));
            if (!rok) E[i] = d[1] / d[0];
          }
          record_pair(ctx, S, seg, t, E[0], NAN, NAN, nullptr, NAN, 7);
          S.rep.nrestarts += 1;
          seg += 1;
          inv[0] = inv[1] = 1.0;
          break;
        }
        const double Enew[2] = {w[0], w[1]};
        const double dE = std::fabs(Enew[0] - E[0]);
        // S130a and S130b are decided by the step's coefficients: the updated
        // vectors are k times the two lowest Ritz vectors, orthonormal in the
        // overlap metric, so |x_{t+1}| = |k|.  Their restart takes the Ritz
        // vectors from the basis: the same vectors in exact arithmetic, but
        // without the cancellation x_t + B y ~ 0 the update suffers when
        // |k| << 1, which would leave X inconsistent with H x.
        {
          const double kn[2] = {std::fabs(cf.k[0]), std::fabs(cf.k[1])};
          const bool a_ = (std::fabs(cf.B[0][0]) < S.o.b_th || std::fabs(cf.B[1][1]) < S.o.b_th) &&
                          dE < S.o.eps1;                                          // S130a
          const bool b_ = kn[0] < S.o.x_th1 || kn[1] < S.o.x_th1 || kn[0] > S.o.x_th2 ||
                          kn[1] > S.o.x_th2;                                      // S130b
          if (phase != SBCI_F64 && (kn[0] < S.o.x_th1 || kn[1] < S.o.x_th1)) {
            // a low-precision phase hands over from the current pair instead:
            // its Ritz problem carries the low-precision images' error,
            // amplified by the near-dependence that makes |k| small
            record_pair(ctx, S, seg, t, Enew[0], dE, NAN, &cf, kn[0], 9);
            SBCI_TRY(next_phase());  // normalises x, recomputes X and E
            inv[0] = inv[1] = 1.0;
            xn[0] = xn[1] = 1.0;
            seg += 1;
            break;
          }
          if (a_ || b_) {
            for (int i = 0; i < 2; ++i) {
              double c1[6];
              for (int k = 0; k < m; ++k) c1[k] = Vp[k * r + i];
              SBCI_TRY(lincomb<double>(ctx, n, P.s[i], basis, c1, m, 0.0));
              SBCI_TRY(lincomb<double>(ctx, n, P.S[i], img, c1, m, 0.0));
            }
            for (int i = 0; i < 2; ++i) {
              std::swap(P.x[i], P.s[i]);
              std::swap(P.X[i], P.S[i]);
              E[i] = Enew[i];
              const double *bs[1] = {P.x[i]};
              double d;
              SBCI_TRY(dots_h(ctx, P, n, P.x[i], bs, 1, &d));
              if (!(d > 0) || !std::isfinite(d))
                return set_error(SBCI_ENUMERIC, "SBCI2: vanishing Ritz vector");
              SBCI_TRY(scale2(ctx, S, P.x[i], 1.0 / std::sqrt(d)));
              SBCI_TRY(scale2(ctx, S, P.X[i], 1.0 / std::sqrt(d)));
            }
            inv[0] = inv[1] = 1.0;
            xn[0] = xn[1] = 1.0;  // the acceptance below rescales by 1 / xn
            SBCI_TRY(pair_residuals(ctx, S, P, E, inv, alpha == 0 ? E[0] : S.Ec[0], dz2));
            const double dz = std::sqrt(dz2[0]);
            if (!std::isfinite(dz)) return set_error(SBCI_ENUMERIC, "SBCI2: non-finite residual");
            int reason = a_ ? 2 : 3;
            const bool ho = hand_over(E[0], dE, dz);
            if (phase == SBCI_F64 && dE < S.o.eps0 && dz < S.o.r0) {            // S127
              conv = true;
              reason = 1;
            } else if (ho) {
              reason = 8;
            }
            record_pair(ctx, S, seg, t, E[0], dE, dz, &cf, kn[0], reason);
            if (conv) break;
            if (reason == 8) {
              SBCI_TRY(next_phase());
              seg += 1;
              break;  // back to the segment start in the new precision
            }
            if (steps >= S.o.max_steps) {
              capped = true;
              S.any_noconv = true;
              break;
            }
            // back to the segment start, with the residuals just formed
            S.rep.nrestarts += 1;
            seg += 1;
            t = 0;
            continue;
          }
        }
        // Eqs. S94-S97 (t = 0: y = A x - C z, x = x + y) and S122-S125
        const double beta = t == 0 ? 0.0 : 1.0;
        for (int i = 0; i < 2; ++i) {
          const int o_ = 1 - i;
          const double Ao = i == 0 ? cf.A01 : cf.A10;
          const double *in1[3] = {z[0], z[1], P.x[o_]};
          const double *in2[3] = {Z[0], Z[1], P.X[o_]};
          double c3[3] = {-cf.C[i][0], -cf.C[i][1], Ao};
          SBCI_TRY(lincomb<double>(ctx, n, P.y[i], in1, c3, 3, beta));
          SBCI_TRY(lincomb<double>(ctx, n, P.Y[i], in2, c3, 3, beta));
        }
        for (int i = 0; i < 2; ++i) {
          const double *in1[2] = {P.y[0], P.y[1]};
          const double *in2[2] = {P.Y[0], P.Y[1]};
          double c2[2] = {cf.B[i][0], cf.B[i][1]};
          SBCI_TRY(lincomb<double>(ctx, n, P.x[i], in1, c2, 2, 1.0));
          SBCI_TRY(lincomb<double>(ctx, n, P.X[i], in2, c2, 2, 1.0));
        }
        for (int i = 0; i < 2; ++i) {
          const double *bs[1] = {P.x[i]};
          double d;
          SBCI_TRY(dots_h(ctx, P, n, P.x[i], bs, 1, &d));
          xn[i] = std::sqrt(d);
          inv[i] = 1.0 / xn[i];
        }
        SBCI_TRY(pair_residuals(ctx, S, P, Enew, inv, alpha == 0 ? Enew[0] : S.Ec[0], dz2));
        const double dz = std::sqrt(dz2[0]);
        if (!std::isfinite(dz) || !std::isfinite(xn[0]) || !std::isfinite(xn[1]) ||
            !std::isfinite(Enew[0]))
          return set_error(SBCI_ENUMERIC, "SBCI2: non-finite residual or norm");
        int reason = 0;
        if (phase == SBCI_F64 && dE < S.o.eps0 && dz < S.o.r0) {                // S127
          conv = true;
          reason = 1;
        } else if (hand_over(Enew[0], dE, dz)) {
          reason = 8;
        } else {
          const bool c_ = dz > S.o.r1 && t > 0;                                   // S130c
          const bool cap = t + 1 >= max_cycle2;
          reason = c_ ? 4 : cap ? 5 : 0;
        }
        record_pair(ctx, S, seg, t, Enew[0], dE, dz, &cf, xn[0], reason);
        E[0] = Enew[0];
        E[1] = Enew[1];
        if (conv) break;
        if (reason == 8) {
          SBCI_TRY(next_phase());  // normalises x, recomputes X and E
          inv[0] = inv[1] = 1.0;
          xn[0] = xn[1] = 1.0;
          seg += 1;
          break;  // back to the segment start in the new precision
        }
        if (steps >= S.o.max_steps) {
          capped = true;
          S.any_noconv = true;
          break;
        }
        if (reason >= 2) {
          // restart (Section S2.5): normalised x, X; the residuals just formed
          // are those of the normalised vectors; back to the segment start
          for (int i = 0; i < 2; ++i) {
            SBCI_TRY(scale2(ctx, S, P.x[i], inv[i]));
            SBCI_TRY(scale2(ctx, S, P.X[i], inv[i]));
          }
          inv[0] = inv[1] = 1.0;
          S.rep.nrestarts += 1;
          seg += 1;
          t = 0;
          continue;
        }
        t += 1;
      }
    }
    // accept state alpha (Algorithm 2); the partner starts the next pair
    double *xc = nullptr;
    SBCI_HIP(hipMalloc(&xc, sizeof(double) * n));
    S.alloc_bytes += sizeof(double) * n;
    SBCI_TRY((convert<double, double>(ctx, n, xc, P.x[0], 1.0 / xn[0])));
    S.xc64.push_back(xc);
    if (first_phase != SBCI_F64) {  // FP32 copy for the low phases' deflation
      float *x32 = nullptr;
      SBCI_HIP(hipMalloc(&x32, sizeof(float) * n));
      S.alloc_bytes += sizeof(float) * n;
      SBCI_TRY((convert<float, double>(ctx, n, x32, xc, 1.0)));
      S.xc32.push_back(x32);
    }
    if (!S.o.s78_printed) {  // the carried image of the accepted root (Eq. S78 reading)
      double *hxc = nullptr;
      SBCI_HIP(hipMalloc(&hxc, sizeof(double) * n));
      S.alloc_bytes += sizeof(double) * n;
      S.Hxc64.push_back(hxc);
      SBCI_TRY((convert<double, double>(ctx, n, hxc, P.X[0], 1.0 / xn[0])));
    }
    S.Ec.push_back(E[0]);
    S.rep.t_converged[std::min(alpha, 15)] = now_s() - S.t0;
    S.rep.resid[std::min(alpha, 15)] = std::sqrt(dz2[0]);
    S.rep.nroots_converged = (int)S.Ec.size();
    SBCI_TRY(scale2(ctx, S, P.x[1], 1.0 / xn[1]));
    SBCI_TRY(scale2(ctx, S, P.X[1], 1.0 / xn[1]));
    std::swap(P.x[0], P.x[1]);
    std::swap(P.X[0], P.X[1]);
    if (alpha + 2 < nroots) {
      // Section S2.2: the next start vector, orthogonalised against the
      // converged roots and against x_0^alpha
      SBCI_TRY(start_vector(ctx, P.k, P.idx, P.U, alpha + 2, P.x[1], P.X[1], S.rep.nsigma_f64));
      SBCI_TRY(project_off(ctx, S, P, P.x[1], P.X[1]));
      const double *bs[1] = {P.x[1]};
      double pa;
      SBCI_TRY(dots_h(ctx, P, n, P.x[0], bs, 1, &pa));
      const double *a1[1] = {P.x[0]}, *a2[1] = {P.X[0]};
      double cfa[1] = {-pa};
      SBCI_TRY(lincomb<double>(ctx, n, P.x[1], a1, cfa, 1, 1.0));
      SBCI_TRY(lincomb<double>(ctx, n, P.X[1], a2, cfa, 1, 1.0));
    }
    if (capped) break;
  }
  // the highest state with SBCI1 (Fig. 1B)
  S.phase = SBCI_F64;
  if ((int)S.Ec.size() < nroots) {
    S.alpha = (int)S.Ec.size();
    if (nroots >= 2) {
      xa = P.x[0];
      Xa = P.X[0];
      SBCI_TRY((convert<double, double>(ctx, n, S.v64[X_], xa, 1.0)));
      SBCI_TRY((convert<double, double>(ctx, n, S.v64[XX_], Xa, 1.0)));
      const double *bs[2] = {S.v64[X_], S.v64[XX_]};
      double d[2];
      SBCI_TRY(dots_h(ctx, P, n, S.v64[X_], bs, 2, d));
      S.E = d[1] / d[0];
    } else {
      SBCI_TRY(initial_vector(ctx, S));
    }
    if (first_phase != SBCI_F64) {
      // SBCI1 with its own precision ladder (as for every later root there)
      SBCI_TRY((convert<float, double>(ctx, n, S.v32[X_], S.v64[X_], 1.0)));
      SBCI_TRY((convert<float, double>(ctx, n, S.v32[XX_], S.v64[XX_], 1.0)));
      S.phase = first_phase;
      SBCI_TRY(start_root<float>(ctx, S));
    } else {
      SBCI_TRY(start_root<double>(ctx, S));
    }
    while (!S.done) {
      if (S.phase == SBCI_F64)
        SBCI_TRY(step_t<double>(ctx, S, nullptr));
      else
        SBCI_TRY(step_t<float>(ctx, S, nullptr));
    }
  } else {
    S.done = true;
  }
  S.alloc_bytes += P.bytes;
  return solver_finish(ctx, energies, dev_vecs, rep_out);
}

}  // namespace sbci
