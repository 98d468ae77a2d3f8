// C ABI of libsbci.so (declared in include/sbci.h): argument validation,
// error reporting and context life cycle.
#include "internal.h"

#include <cmath>
#include <cstring>

namespace sbci {

int solver_begin(sbci_ctx *ctx, int nroots, double tol, const sbci_opts *opt);
int solver_iterate(sbci_ctx *ctx, double *dev_x);
int solver_step(sbci_ctx *ctx, sbci_step_info *info, int *done);
int solver_finish(sbci_ctx *ctx, double *energies, double *dev_vecs, sbci_report *rep);
void solver_free(sbci_ctx *ctx);
int davidson(sbci_ctx *ctx, int nroots, double tol, const sbci_opts *opt, double *energies,
             double *dev_vecs, sbci_report *rep);
int sbci2_solve(sbci_ctx *ctx, int nroots, double tol, const sbci_opts *opt, double *energies,
                double *dev_vecs, sbci_report *rep);

namespace {
thread_local std::string g_err;
}

int set_error(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

int ensure(Workspace &w, size_t bytes) {
  if (w.bytes >= bytes && w.ptr) return SBCI_OK;
  if (w.ptr) hipFree(w.ptr);
  w.ptr = nullptr;
  w.bytes = 0;
  hipError_t e = hipMalloc(&w.ptr, bytes);
  if (e != hipSuccess) {
    w.ptr = nullptr;
    return set_error(SBCI_ENOMEM, std::string("workspace hipMalloc: ") + hipGetErrorString(e));
  }
  w.bytes = bytes;
  return SBCI_OK;
}

namespace {

int validate_integrals(int n, const double *h1, const double *eri) {
  double hmax = 0, gmax = 0;
  for (int i = 0; i < n * n; ++i) hmax = std::fmax(hmax, std::fabs(h1[i]));
  const size_t n4 = (size_t)n * n * n * n;
  for (size_t i = 0; i < n4; ++i) {
    if (!std::isfinite(eri[i])) return set_error(SBCI_EINVAL, "eri has a non-finite entry");
    gmax = std::fmax(gmax, std::fabs(eri[i]));
  }
  for (int i = 0; i < n * n; ++i)
    if (!std::isfinite(h1[i])) return set_error(SBCI_EINVAL, "h1 has a non-finite entry");
  const double th = 1e-12 * std::fmax(hmax, 1e-300), tg = 1e-12 * std::fmax(gmax, 1e-300);
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q)
      if (std::fabs(h1[p * n + q] - h1[q * n + p]) > th)
        return set_error(SBCI_EINVAL, "h1 is not symmetric");
  auto G = [&](int p, int q, int r, int s) { return eri[(((size_t)p * n + q) * n + r) * n + s]; };
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q)
      for (int r = 0; r < n; ++r)
        for (int s = 0; s < n; ++s) {
          const double v = G(p, q, r, s);
          if (std::fabs(v - G(q, p, r, s)) > tg || std::fabs(v - G(p, q, s, r)) > tg ||
              std::fabs(v - G(r, s, p, q)) > tg)
            return set_error(SBCI_EINVAL, "eri lacks the 8-fold permutational symmetry");
        }
  return SBCI_OK;
}

int64_t choose(int n, int k) {
  if (k < 0 || k > n) return 0;
  long double r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return (int64_t)(r + 0.5L);
}

}  // namespace
}  // namespace sbci

using namespace sbci;

extern "C" {

void sbci_default_opts(sbci_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->eps0 = 1e-10;
  o->r0 = 1e-5;
  o->b_th = 1e-2;
  o->eps1 = 1e-7;
  o->x_th1 = 0.1;
  o->x_th2 = 1.2;
  o->r1 = 1.0;
  o->max_cycle = 20;
  o->max_steps = 2000;
  o->precision = SBCI_F64;
  o->mix_eps0 = 1e-8;
  o->mix_r0 = 1e-3;
  o->mix_stall = 3;
  o->precond_floor = 1e-8;
  o->lindep = 1e-14;
  o->max_space = 0;
  o->x0 = nullptr;
  o->bf16_eps0 = 1e-5;
  o->bf16_r0 = 1e-2;
  o->max_cycle2 = 10;
  o->s78_printed = 0;
}

const char *sbci_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace sbci {
// Context on a given stream; own_stream = false leaves the stream to the caller
// (the batch form builds many contexts on one stream).
int create_context(int norb, int nalpha, int nbeta, const double *h1, const double *eri,
                   hipStream_t stream, bool own_stream, sbci_ctx **out, const int *orbsym,
                   int irrep) {
  if (!out) return set_error(SBCI_EINVAL, "out is NULL");
  *out = nullptr;
  if (norb < 1 || norb > 63) return set_error(SBCI_EINVAL, "norb must be in [1, 63]");
  if (nalpha < 0 || nbeta < 0 || nalpha > norb || nbeta > norb)
    return set_error(SBCI_EINVAL, "nalpha and nbeta must be in [0, norb]");
  if (!h1 || !eri) return set_error(SBCI_EINVAL, "h1 or eri is NULL");
  const int64_t nsa = choose(norb, nalpha), nsb = choose(norb, nbeta);
  if (nsa > (int64_t)1 << 30 || nsb > (int64_t)1 << 30)
    return set_error(SBCI_EINVAL, "string space too large for 32-bit string addresses");
  SBCI_TRY(validate_integrals(norb, h1, eri));
  int dev = 0;
  SBCI_HIP(hipGetDevice(&dev));
  sbci_ctx *ctx = new sbci_ctx();
  ctx->norb = norb;
  ctx->na = nalpha;
  ctx->nb = nbeta;
  ctx->device = dev;
  if (own_stream) {
    hipError_t e = hipStreamCreateWithFlags(&ctx->own_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete ctx;
      return set_error(SBCI_EDEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
    }
    ctx->stream = ctx->own_stream;
  } else {
    ctx->stream = stream;
  }
  int rc = build_tables(ctx, h1, eri);
  if (rc == SBCI_OK && orbsym) rc = setup_symmetry(ctx, orbsym, irrep, h1, eri);
  if (rc != SBCI_OK) {
    std::string msg = g_err;
    sbci_destroy(ctx);
    return set_error(rc, msg);
  }
  *out = ctx;
  return SBCI_OK;
}
}  // namespace sbci

extern "C" {

int sbci_create(int norb, int nalpha, int nbeta, const double *h1, const double *eri,
                sbci_ctx **out) {
  return create_context(norb, nalpha, nbeta, h1, eri, nullptr, true, out);
}

int sbci_create_sym(int norb, int nalpha, int nbeta, const double *h1, const double *eri,
                    const int *orbsym, int irrep, sbci_ctx **out) {
  if (!orbsym) return set_error(SBCI_EINVAL, "orbsym is NULL");
  return create_context(norb, nalpha, nbeta, h1, eri, nullptr, true, out, orbsym, irrep);
}

int sbci_sym_blocks(const sbci_ctx *ctx, int64_t *out) {
  if (!ctx || !out) return set_error(SBCI_EINVAL, "NULL argument");
  return sym_blocks(ctx, out);
}

int sbci_destroy(sbci_ctx *ctx) {
  if (!ctx) return SBCI_OK;
  hipStreamSynchronize(ctx->stream);
  solver_free(ctx);
  free_symmetry(ctx);
  free_tables(ctx);
  hipFree(ctx->ws_t.ptr);
  hipFree(ctx->ws_s.ptr);
  hipFree(ctx->ws_red.ptr);
  hipFree(ctx->ws_q.ptr);
  hipFree(ctx->ws_rmax.ptr);
  if (ctx->own_stream) hipStreamDestroy(ctx->own_stream);
  delete ctx;
  return SBCI_OK;
}

int sbci_set_stream(sbci_ctx *ctx, void *stream) {
  if (!ctx) return set_error(SBCI_EINVAL, "ctx is NULL");
  SBCI_HIP(hipStreamSynchronize(ctx->stream));
  ctx->stream = static_cast<hipStream_t>(stream);  // NULL: the null (legacy default) stream
  return SBCI_OK;
}

int64_t sbci_ndet(const sbci_ctx *ctx) { return ctx ? ctx->ndet : -1; }

int64_t sbci_nstrings(const sbci_ctx *ctx, int spin) {
  if (!ctx) return -1;
  return spin == 0 ? ctx->A.ns : ctx->B.ns;
}

int sbci_tables(sbci_ctx *ctx, int which, void *dev_out, int64_t *bytes) {
  if (!ctx) return set_error(SBCI_EINVAL, "ctx is NULL");
  const SpinTables &T = (which == 0 || which == 2) ? ctx->A : ctx->B;
  const void *src = nullptr;
  int64_t nb = 0;
  switch (which) {
    case 0:
    case 1:
      src = T.str;
      nb = (int64_t)sizeof(uint64_t) * T.ns;
      break;
    case 2:
    case 3:
      src = T.tab;
      nb = (int64_t)sizeof(Ent) * T.ns * T.s;
      break;
    default:
      return set_error(SBCI_EINVAL, "which must be 0..3");
  }
  if (bytes) *bytes = nb;
  if (dev_out && nb > 0) {
    SBCI_HIP(hipMemcpyAsync(dev_out, src, nb, hipMemcpyDeviceToDevice, ctx->stream));
    SBCI_HIP(hipStreamSynchronize(ctx->stream));
  }
  return SBCI_OK;
}

int sbci_hdiag(sbci_ctx *ctx, double *dev_out) {
  if (!ctx || !dev_out) return set_error(SBCI_EINVAL, "NULL argument");
  SBCI_HIP(hipMemcpyAsync(dev_out, ctx->hdiag, sizeof(double) * ctx->ndet, hipMemcpyDeviceToDevice,
                          ctx->stream));
  return SBCI_OK;
}

int sbci_sigma(sbci_ctx *ctx, const void *dev_c, void *dev_sigma, int nvec, int dtype) {
  if (!ctx || !dev_c || !dev_sigma) return set_error(SBCI_EINVAL, "NULL argument");
  if (nvec < 1 || nvec > 65535) return set_error(SBCI_EINVAL, "nvec must be in [1, 65535]");
  if (dtype != SBCI_F64 && dtype != SBCI_F32 && dtype != SBCI_BF16)
    return set_error(SBCI_EINVAL, "unknown dtype");
  const size_t es = dtype == SBCI_F64 ? 8 : 4;
  const char *a = static_cast<const char *>(dev_c), *b = static_cast<const char *>(dev_sigma);
  const size_t span = es * (size_t)ctx->ndet * nvec;
  if (a < b + span && b < a + span) return set_error(SBCI_EINVAL, "c and sigma overlap");
  return sigma(ctx, dev_c, dev_sigma, nvec, dtype);
}

int sbci_sigma_noalloc(sbci_ctx *ctx, const void *dev_c, void *dev_sigma, int nvec, int dtype) {
  if (!ctx || !dev_c || !dev_sigma) return set_error(SBCI_EINVAL, "NULL argument");
  if (nvec < 1 || nvec > 65535) return set_error(SBCI_EINVAL, "nvec must be in [1, 65535]");
  if (dtype != SBCI_F64 && dtype != SBCI_F32 && dtype != SBCI_BF16)
    return set_error(SBCI_EINVAL, "unknown dtype");
  const size_t es = dtype == SBCI_F64 ? 8 : 4;
  const char *a = static_cast<const char *>(dev_c), *b = static_cast<const char *>(dev_sigma);
  const size_t span = es * (size_t)ctx->ndet * nvec;
  if (a < b + span && b < a + span) return set_error(SBCI_EINVAL, "c and sigma overlap");
  return sigma_noalloc(ctx, dev_c, dev_sigma, nvec, dtype);
}

int sbci_sigma_timed(sbci_ctx *ctx, const void *dev_c, void *dev_sigma, int nvec, int dtype,
                     float *ms_parts) {
  if (!ms_parts) return set_error(SBCI_EINVAL, "ms_parts is NULL");
  if (!ctx || !dev_c || !dev_sigma) return set_error(SBCI_EINVAL, "NULL argument");
  if (nvec < 1 || nvec > 65535) return set_error(SBCI_EINVAL, "nvec must be in [1, 65535]");
  if (dtype != SBCI_F64 && dtype != SBCI_F32 && dtype != SBCI_BF16)
    return set_error(SBCI_EINVAL, "unknown dtype");
  return sigma_profile(ctx, dev_c, dev_sigma, nvec, dtype, ms_parts);
}

int sbci_set_deterministic(sbci_ctx *ctx, int on) {
  if (!ctx) return set_error(SBCI_EINVAL, "ctx is NULL");
  if (on != 0 && on != 1) return set_error(SBCI_EINVAL, "on must be 0 or 1");
  ctx->deterministic = on != 0;
  return SBCI_OK;
}

int sbci_set_opp_form(sbci_ctx *ctx, int form) {
  if (!ctx) return set_error(SBCI_EINVAL, "ctx is NULL");
  if (form != SBCI_OPP_AUTO && form != SBCI_OPP_PAIR && form != SBCI_OPP_ORBITAL &&
      form != SBCI_OPP_ORBITAL_WINDOWED && form != SBCI_OPP_CLASS_MFMA)
    return set_error(SBCI_EINVAL, "unknown opposite-spin form");
  if (form == SBCI_OPP_CLASS_MFMA && !ctx->sym)
    return set_error(SBCI_EINVAL, "the class MFMA form is for symmetry-blocked contexts");
  if ((form == SBCI_OPP_ORBITAL || form == SBCI_OPP_ORBITAL_WINDOWED) && ctx->sym)
    return set_error(SBCI_EINVAL, "symmetry-blocked contexts have no orbital form");
  ctx->opp_form = form;
  return SBCI_OK;
}

int sbci_get_opp_form(sbci_ctx *ctx, int dtype, int *form) {
  if (!ctx || !form) return set_error(SBCI_EINVAL, "NULL argument");
  if (dtype != SBCI_F64 && dtype != SBCI_F32 && dtype != SBCI_BF16)
    return set_error(SBCI_EINVAL, "unknown dtype");
  return opp_form(ctx, dtype, form);
}

int sbci_set_same_form(sbci_ctx *ctx, int form) {
  if (!ctx) return set_error(SBCI_EINVAL, "ctx is NULL");
  if (form != SBCI_SAME_AUTO && form != SBCI_SAME_LISTS && form != SBCI_SAME_DENSE)
    return set_error(SBCI_EINVAL, "unknown same-spin form");
  ctx->same_form = form;
  return SBCI_OK;
}

int sbci_get_same_form(sbci_ctx *ctx, int spin, int dtype, int *form) {
  if (!ctx || !form) return set_error(SBCI_EINVAL, "NULL argument");
  if (spin != 0 && spin != 1) return set_error(SBCI_EINVAL, "spin must be 0 or 1");
  if (dtype != SBCI_F64 && dtype != SBCI_F32 && dtype != SBCI_BF16)
    return set_error(SBCI_EINVAL, "unknown dtype");
  return same_form(ctx, spin, dtype, form);
}

int sbci_begin(sbci_ctx *ctx, int nroots, double tol, const sbci_opts *opt) {
  if (!ctx) return set_error(SBCI_EINVAL, "ctx is NULL");
  return solver_begin(ctx, nroots, tol, opt);
}

int sbci_step(sbci_ctx *ctx, sbci_step_info *info, int *done) {
  if (!ctx) return set_error(SBCI_EINVAL, "ctx is NULL");
  return solver_step(ctx, info, done);
}

int sbci_finish(sbci_ctx *ctx, double *energies, double *dev_vecs, sbci_report *rep) {
  if (!ctx) return set_error(SBCI_EINVAL, "ctx is NULL");
  return solver_finish(ctx, energies, dev_vecs, rep);
}

int sbci_iterate(sbci_ctx *ctx, double *dev_x) {
  if (!ctx || !dev_x) return set_error(SBCI_EINVAL, "NULL argument");
  return solver_iterate(ctx, dev_x);
}

int sbci_solve(sbci_ctx *ctx, int nroots, double tol, const sbci_opts *opt, double *energies,
               double *dev_vecs, sbci_report *rep) {
  if (!ctx || !energies) return set_error(SBCI_EINVAL, "NULL argument");
  SBCI_TRY(solver_begin(ctx, nroots, tol, opt));
  int done = 0;
  while (!done) SBCI_TRY(solver_step(ctx, nullptr, &done));
  return solver_finish(ctx, energies, dev_vecs, rep);
}

int sbci_set_trace(sbci_ctx *ctx, int on) {
  if (!ctx) return set_error(SBCI_EINVAL, "ctx is NULL");
  ctx->trace_on = on != 0;
  return SBCI_OK;
}

int sbci_set_progress(sbci_ctx *ctx, sbci_progress_fn fn, void *user) {
  if (!ctx) return set_error(SBCI_EINVAL, "ctx is NULL");
  ctx->progress = fn;
  ctx->progress_user = user;
  return SBCI_OK;
}

int sbci_trace(sbci_ctx *ctx, sbci_step_info *out, int max) {
  if (!ctx) return set_error(SBCI_EINVAL, "ctx is NULL");
  int n = (int)std::min<size_t>(ctx->trace.size(), max > 0 ? (size_t)max : 0);
  if (out)
    for (int i = 0; i < n; ++i) out[i] = ctx->trace[i];
  return out ? n : (int)ctx->trace.size();
}

int sbci_davidson(sbci_ctx *ctx, int nroots, double tol, const sbci_opts *opt, double *energies,
                  double *dev_vecs, sbci_report *rep) {
  if (!ctx || !energies) return set_error(SBCI_EINVAL, "NULL argument");
  solver_free(ctx);  // an earlier step-level solve ends here (its state is not Davidson's)
  return davidson(ctx, nroots, tol, opt, energies, dev_vecs, rep);
}

int sbci_solve2(sbci_ctx *ctx, int nroots, double tol, const sbci_opts *opt, double *energies,
                double *dev_vecs, sbci_report *rep) {
  if (!ctx || !energies) return set_error(SBCI_EINVAL, "NULL argument");
  return sbci2_solve(ctx, nroots, tol, opt, energies, dev_vecs, rep);
}

}  // extern "C"
