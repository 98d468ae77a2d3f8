// Vector passes of the SBCI step with FP64 reductions (HBM-bound kernels).
//
// k_update is the fused symplectic-Euler pass of one SBCI1 step:
//   y <- sy*y - c*z,  Y <- sy*Y - c*Z            (Eqs. S25-S26 / S56-S57)
//   x <- sx*x + b*y,  X <- sx*X + b*Y            (Eqs. S27-S28 / S58-S59)
//   z' = (X - E x) * inv_norm                     (Eq. S60; Algorithm 1's residual)
//   w  = z' / (D - E0)                            (Eq. S31 before the projection)
// and reduces, in FP64, every inner product the next step's Ritz problem
// needs except those involving Z = H z (which exists only after the next
// sigma): |z'|^2, x.x, x.y, y.y, x.X, x.Y, y.Y, optionally x.w, y.w, w.w, and
// the projections x_c^i . w on the converged roots.  sx rescales x, X at the
// start of a segment (a restart normalises x without a separate pass) and
// sy = 0 drops y, Y (y_0 = 0 at a segment start).
//
// Reductions are deterministic: each block writes its partial sums and a
// one-block kernel adds the partials in a fixed order.
#include "internal.h"

namespace sbci {

namespace {

constexpr int BS = 256;
constexpr int MAXQ = 48;
// blocks of a vector pass (grid-stride beyond): measured on MI355X with a
// 7-read / 5-write FP64 stream of 165.6 M elements, 16384 blocks of 256
// threads with 4 elements in flight per thread reach 5.15 TB/s against
// 4.63 TB/s with 2048 blocks and 2 elements (a plain copy reaches 5.6 TB/s)
constexpr int kMaxBlocks = 16384;
constexpr int MAXV = 16;

struct Ptrs {
  const void *p[MAXV];
};

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Reduce v[0..nq) over the block and store the block's partial sums;
// k_reduce (launched next on the same stream) adds the partials of all
// blocks in a fixed order.  The kernel boundary orders the two, so no
// device-scope fence is needed (on this multi-XCD part such a fence writes
// back and invalidates L2, which starves the streaming passes).
template <int NQ>
__device__ void grid_reduce(double (&v)[NQ], int nq, double *__restrict__ part, unsigned *,
                            double *) {
  __shared__ double sh[BS / 64][NQ];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    if (q >= nq) break;
    double s = wave_sum(v[q]);
    if (lane == 0) sh[wave][q] = s;
  }
  __syncthreads();
  if (threadIdx.x < nq) {
    double s = 0;
    for (int w = 0; w < BS / 64; ++w) s += sh[w][threadIdx.x];
    part[(size_t)blockIdx.x * MAXQ + threadIdx.x] = s;
  }
}

// out[q] = sum over blocks b (in order b = t, t + BS, ... per thread t, then
// a fixed tree) of part[b][q].
__global__ __launch_bounds__(BS) void k_reduce(const double *__restrict__ part, unsigned nblocks,
                                               int nq, double *__restrict__ out) {
  __shared__ double sh[BS / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int q = 0; q < nq; ++q) {
    double s = 0;
    for (unsigned b = threadIdx.x; b < nblocks; b += BS) s += part[(size_t)b * MAXQ + q];
    s = wave_sum(s);
    if (lane == 0) sh[wave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0;
      for (int w = 0; w < BS / 64; ++w) t += sh[w];
      out[q] = t;
    }
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(BS) void k_dots(int64_t n, const T *__restrict__ a, Ptrs bs, int nb,
                                             double *part, unsigned *ticket, double *out) {
  constexpr int U = 2;
  double v[MAXV];
#pragma unroll
  for (int q = 0; q < MAXV; ++q) v[q] = 0;
  const int64_t S = (int64_t)gridDim.x * BS;
  int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  for (; i + (U - 1) * S < n; i += U * S) {
    double ai[U];
#pragma unroll
    for (int u = 0; u < U; ++u) ai[u] = (double)a[i + u * S];
#pragma unroll
    for (int q = 0; q < MAXV; ++q)
      if (q < nb) {
        const T *bq = static_cast<const T *>(bs.p[q]);
#pragma unroll
        for (int u = 0; u < U; ++u) v[q] += ai[u] * (double)bq[i + u * S];
      }
  }
  for (; i < n; i += S) {
    const double ai = (double)a[i];
#pragma unroll
    for (int q = 0; q < MAXV; ++q)
      if (q < nb) v[q] += ai * (double)static_cast<const T *>(bs.p[q])[i];
  }
  grid_reduce<MAXV>(v, nb, part, ticket, out);
}

struct Coefs {
  double c[MAXV];
};

template <typename T>
__global__ __launch_bounds__(BS) void k_lincomb(int64_t n, T *__restrict__ out, Ptrs xs, Coefs cf,
                                                int nx, double beta) {
  constexpr int U = 4;
  const int64_t S = (int64_t)gridDim.x * BS;
  int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  for (; i + (U - 1) * S < n; i += U * S) {
    double s[U];
#pragma unroll
    for (int u = 0; u < U; ++u) s[u] = beta == 0.0 ? 0.0 : beta * (double)out[i + u * S];
#pragma unroll
    for (int q = 0; q < MAXV; ++q)
      if (q < nx) {
        const T *xq = static_cast<const T *>(xs.p[q]);
#pragma unroll
        for (int u = 0; u < U; ++u) s[u] += cf.c[q] * (double)xq[i + u * S];
      }
#pragma unroll
    for (int u = 0; u < U; ++u) out[i + u * S] = (T)s[u];
  }
  for (; i < n; i += S) {
    double s = beta == 0.0 ? 0.0 : beta * (double)out[i];
#pragma unroll
    for (int q = 0; q < MAXV; ++q)
      if (q < nx) s += cf.c[q] * (double)static_cast<const T *>(xs.p[q])[i];
    out[i] = (T)s;
  }
}

template <typename Td, typename Ts>
__global__ __launch_bounds__(BS) void k_convert(int64_t n, Td *__restrict__ dst,
                                                const Ts *__restrict__ src, double scale) {
  constexpr int U = 4;
  const int64_t S = (int64_t)gridDim.x * BS;
  int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  for (; i + (U - 1) * S < n; i += U * S) {
    Ts v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = src[i + u * S];
#pragma unroll
    for (int u = 0; u < U; ++u) dst[i + u * S] = (Td)(scale * (double)v[u]);
  }
  for (; i < n; i += S) dst[i] = (Td)(scale * (double)src[i]);
}

// NC: compile-time bound on the number of converged roots (a bucket of
// a.nconv), so that only that many projection loads are kept in flight.
template <typename T, int NC>
__global__ __launch_bounds__(BS) void k_update(int64_t n, T *__restrict__ x, T *__restrict__ X,
                                               T *__restrict__ y, T *__restrict__ Y,
                                               const T *__restrict__ z, const T *__restrict__ Z,
                                               T *__restrict__ w, const T *__restrict__ D, Ptrs xc,
                                               UpdateArgs a, double *part, unsigned *ticket,
                                               double *out) {
  // slots: 0 |z'|^2, 1 xx, 2 xy, 3 yy, 4 xX, 5 xY, 6 yY, 7 xw, 8 yw, 9 ww, 10+j xc_j.w
  constexpr int U = 4;
  double v[10 + NC];
#pragma unroll
  for (int q = 0; q < 10 + NC; ++q) v[q] = 0;
  const double b = a.b, c = a.c, E = a.E, inv = a.inv_norm, E0 = a.E0, fl = a.floor, sx = a.sx;
  const int64_t S = (int64_t)gridDim.x * BS;
  auto element = [&](int64_t k, double zi, double Zi, double yi, double Yi, double xi, double Xi,
                     double Di) {
    const double yn = yi - c * zi, Yn = Yi - c * Zi;
    const double xn = sx * xi + b * yn, Xn = sx * Xi + b * Yn;
    const double r = (Xn - E * xn) * inv;
    double den = Di - E0;
    if (fabs(den) < fl) den = fl;
    const double wi = r / den;
    x[k] = (T)xn;
    X[k] = (T)Xn;
    y[k] = (T)yn;
    Y[k] = (T)Yn;
    w[k] = (T)wi;
    // reduce what was stored (the next step sees the rounded vectors)
    const double xs = (double)(T)xn, ys = (double)(T)yn, Xs = (double)(T)Xn, Ys = (double)(T)Yn;
    const double ws = (double)(T)wi;
    v[0] += r * r;
    v[1] += xs * xs;
    v[2] += xs * ys;
    v[3] += ys * ys;
    v[4] += xs * Xs;
    v[5] += xs * Ys;
    v[6] += ys * Ys;
    if (a.want_zdots) {
      v[7] += xs * ws;
      v[8] += ys * ws;
      v[9] += ws * ws;
    }
#pragma unroll
    for (int j = 0; j < NC; ++j)
      if (j < a.nconv) v[10 + j] += ws * (double)static_cast<const T *>(xc.p[j])[k];
  };
  int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  for (; i + (U - 1) * S < n; i += U * S) {
    double zi[U], Zi[U], yi[U], Yi[U], xi[U], Xi[U], Di[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t k = i + u * S;
      zi[u] = a.read_z ? (double)z[k] : 0.0;
      Zi[u] = a.read_z ? (double)Z[k] : 0.0;
      yi[u] = a.sy ? (double)y[k] : 0.0;
      Yi[u] = a.sy ? (double)Y[k] : 0.0;
      xi[u] = (double)x[k];
      Xi[u] = (double)X[k];
      Di[u] = (double)D[k];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) element(i + u * S, zi[u], Zi[u], yi[u], Yi[u], xi[u], Xi[u], Di[u]);
  }
  for (; i < n; i += S)
    element(i, a.read_z ? (double)z[i] : 0.0, a.read_z ? (double)Z[i] : 0.0,
            a.sy ? (double)y[i] : 0.0, a.sy ? (double)Y[i] : 0.0, (double)x[i], (double)X[i],
            (double)D[i]);
  grid_reduce<10 + NC>(v, 10 + a.nconv, part, ticket, out);
}

// Residual pass of one state (SBCI2, Eqs. S98/S100, S126/S128 with Eq.
// S101's preconditioner): r = (X - E x) * inv, w = r / (D - E0) (floored);
// reduces |r|^2 and the projections xc_j . w.
template <typename T, int NC>
__global__ __launch_bounds__(BS) void k_resid(int64_t n, const T *__restrict__ x,
                                              const T *__restrict__ X, const T *__restrict__ D,
                                              double E, double inv, double E0, double fl, Ptrs xc,
                                              int nconv, T *__restrict__ w, double *part,
                                              unsigned *ticket, double *out) {
  constexpr int U = 4;
  double v[1 + NC];
#pragma unroll
  for (int q = 0; q < 1 + NC; ++q) v[q] = 0;
  const int64_t S = (int64_t)gridDim.x * BS;
  auto element = [&](int64_t k, double xi, double Xi, double Di) {
    const double r = (Xi - E * xi) * inv;
    double den = Di - E0;
    if (fabs(den) < fl) den = fl;
    const T wt = (T)(r / den);
    w[k] = wt;
    v[0] += r * r;
    const double ws = (double)wt;
#pragma unroll
    for (int j = 0; j < NC; ++j)
      if (j < nconv) v[1 + j] += ws * (double)static_cast<const T *>(xc.p[j])[k];
  };
  int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  for (; i + (U - 1) * S < n; i += U * S) {
    double xi[U], Xi[U], Di[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      xi[u] = (double)x[i + u * S];
      Xi[u] = (double)X[i + u * S];
      Di[u] = (double)D[i + u * S];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) element(i + u * S, xi[u], Xi[u], Di[u]);
  }
  for (; i < n; i += S) element(i, (double)x[i], (double)X[i], (double)D[i]);
  grid_reduce<1 + NC>(v, 1 + nconv, part, ticket, out);
}

// z = w - sum_j d_j xc_j (in place); reduces x.z, y.z, z.z
template <typename T, int NC>
__global__ __launch_bounds__(BS) void k_deflate(int64_t n, T *__restrict__ w, const T *__restrict__ x,
                                                const T *__restrict__ y, Ptrs xc, int nconv,
                                                const double *__restrict__ d, double *part,
                                                unsigned *ticket, double *out) {
  constexpr int U = 4;
  double dj[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) dj[j] = j < nconv ? d[j] : 0.0;
  double v[3] = {0, 0, 0};
  const int64_t S = (int64_t)gridDim.x * BS;
  auto element = [&](int64_t k, double zi, double xi, double yi) {
#pragma unroll
    for (int j = 0; j < NC; ++j)
      if (j < nconv) zi -= dj[j] * (double)static_cast<const T *>(xc.p[j])[k];
    const T zt = (T)zi;
    w[k] = zt;
    const double zs = (double)zt;
    v[0] += xi * zs;
    v[1] += yi * zs;
    v[2] += zs * zs;
  };
  int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  for (; i + (U - 1) * S < n; i += U * S) {
    double zi[U], xi[U], yi[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      zi[u] = (double)w[i + u * S];
      xi[u] = (double)x[i + u * S];
      yi[u] = (double)y[i + u * S];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) element(i + u * S, zi[u], xi[u], yi[u]);
  }
  for (; i < n; i += S) element(i, (double)w[i], (double)x[i], (double)y[i]);
  grid_reduce<3>(v, 3, part, ticket, out);
}

// x.Z, y.Z, z.Z (H acting on the right-hand vector)
template <typename T>
__global__ __launch_bounds__(BS) void k_dots_xyz(int64_t n, const T *__restrict__ x,
                                                 const T *__restrict__ y, const T *__restrict__ z,
                                                 const T *__restrict__ Z, double *part,
                                                 unsigned *ticket, double *out) {
  constexpr int U = 4;
  double v[3] = {0, 0, 0};
  const int64_t S = (int64_t)gridDim.x * BS;
  int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  for (; i + (U - 1) * S < n; i += U * S) {
    double Zi[U], xi[U], yi[U], zi[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      Zi[u] = (double)Z[i + u * S];
      xi[u] = (double)x[i + u * S];
      yi[u] = (double)y[i + u * S];
      zi[u] = (double)z[i + u * S];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      v[0] += xi[u] * Zi[u];
      v[1] += yi[u] * Zi[u];
      v[2] += zi[u] * Zi[u];
    }
  }
  for (; i < n; i += S) {
    const double Zi = (double)Z[i];
    v[0] += (double)x[i] * Zi;
    v[1] += (double)y[i] * Zi;
    v[2] += (double)z[i] * Zi;
  }
  grid_reduce<3>(v, 3, part, ticket, out);
}

// Overlap and H matrices of an m-vector basis in one pass (the pair steps
// of Algorithm 2, Eqs. S83-S87 / S103-S107): out[q] = b_i . b_j and
// out[P + q] = b_i . h_j (H on the right-hand vector) for the upper
// triangle i <= j in row-major order, P = m (m + 1) / 2, h_j the image of b_j.
template <int M>
__global__ __launch_bounds__(BS) void k_gram(int64_t n, Ptrs b, Ptrs h, double *part,
                                             unsigned *ticket, double *out) {
  constexpr int P = M * (M + 1) / 2;
  double v[2 * P];
#pragma unroll
  for (int q = 0; q < 2 * P; ++q) v[q] = 0;
  const int64_t S = (int64_t)gridDim.x * BS;
  for (int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x; i < n; i += S) {
    double bi[M], hi[M];
#pragma unroll
    for (int a = 0; a < M; ++a) {
      bi[a] = static_cast<const double *>(b.p[a])[i];
      hi[a] = static_cast<const double *>(h.p[a])[i];
    }
    int q = 0;
#pragma unroll
    for (int a = 0; a < M; ++a)
#pragma unroll
      for (int c = a; c < M; ++c, ++q) {
        v[q] += bi[a] * bi[c];
        v[P + q] += bi[a] * hi[c];
      }
  }
  grid_reduce<2 * P>(v, 2 * P, part, ticket, out);
}

unsigned grid_for(int64_t n) {
  int64_t b = (n + BS - 1) / BS;
  if (b > kMaxBlocks) b = kMaxBlocks;
  if (b < 1) b = 1;
  return (unsigned)b;
}

struct RedBuf {
  double *part;
  unsigned *ticket;
};

int red_buf(sbci_ctx *ctx, RedBuf &r) {
  const size_t part_b = sizeof(double) * kMaxBlocks * MAXQ;
  if (!ctx->ws_red.ptr) {
    SBCI_TRY(ensure(ctx->ws_red, part_b + 256));
    SBCI_HIP(hipMemsetAsync(ctx->ws_red.ptr, 0, part_b + 256, ctx->stream));
  }
  r.part = static_cast<double *>(ctx->ws_red.ptr);
  r.ticket = reinterpret_cast<unsigned *>(static_cast<char *>(ctx->ws_red.ptr) + part_b);
  return SBCI_OK;
}

}  // namespace

template <typename T>
int dots(sbci_ctx *ctx, int64_t n, const T *a, const T *const *bs, int nb, double *out) {
  if (nb < 1 || nb > MAXV) return set_error(SBCI_EINVAL, "dots: 1..16 vectors");
  RedBuf r;
  SBCI_TRY(red_buf(ctx, r));
  Ptrs p{};
  for (int i = 0; i < nb; ++i) p.p[i] = bs[i];
  k_dots<T><<<grid_for(n), BS, 0, ctx->stream>>>(n, a, p, nb, r.part, r.ticket, out);
  k_reduce<<<1, BS, 0, ctx->stream>>>(r.part, grid_for(n), nb, out);
  SBCI_CHECK_LAUNCH();
  return SBCI_OK;
}

template <typename T>
int lincomb(sbci_ctx *ctx, int64_t n, T *out, const T *const *xs, const double *coef, int nx,
            double beta) {
  if (nx < 0 || nx > MAXV) return set_error(SBCI_EINVAL, "lincomb: 0..16 vectors");
  Ptrs p{};
  Coefs cf{};
  for (int i = 0; i < nx; ++i) {
    p.p[i] = xs[i];
    cf.c[i] = coef[i];
  }
  k_lincomb<T><<<grid_for(n), BS, 0, ctx->stream>>>(n, out, p, cf, nx, beta);
  SBCI_CHECK_LAUNCH();
  return SBCI_OK;
}

template <typename Td, typename Ts>
int convert(sbci_ctx *ctx, int64_t n, Td *dst, const Ts *src, double scale) {
  k_convert<Td, Ts><<<grid_for(n), BS, 0, ctx->stream>>>(n, dst, src, scale);
  SBCI_CHECK_LAUNCH();
  return SBCI_OK;
}

template <typename T>
int update(sbci_ctx *ctx, int64_t n, T *x, T *X, T *y, T *Y, const T *z, const T *Z, T *w,
           const T *D, const T *const *xc, const UpdateArgs &a, double *out) {
  if (a.nconv < 0 || a.nconv > MAXV) return set_error(SBCI_EINVAL, "update: too many roots");
  RedBuf r;
  SBCI_TRY(red_buf(ctx, r));
  Ptrs p{};
  for (int i = 0; i < a.nconv; ++i) p.p[i] = xc[i];
  if (a.nconv == 0)
    k_update<T, 1><<<grid_for(n), BS, 0, ctx->stream>>>(n, x, X, y, Y, z, Z, w, D, p, a, r.part,
                                                        r.ticket, out);
  else if (a.nconv <= 4)
    k_update<T, 4><<<grid_for(n), BS, 0, ctx->stream>>>(n, x, X, y, Y, z, Z, w, D, p, a, r.part,
                                                        r.ticket, out);
  else
    k_update<T, MAXV><<<grid_for(n), BS, 0, ctx->stream>>>(n, x, X, y, Y, z, Z, w, D, p, a, r.part,
                                                           r.ticket, out);
  k_reduce<<<1, BS, 0, ctx->stream>>>(r.part, grid_for(n), 10 + a.nconv, out);
  SBCI_CHECK_LAUNCH();
  return SBCI_OK;
}

template <typename T>
int deflate(sbci_ctx *ctx, int64_t n, T *w, const T *x, const T *y, const T *const *xc, int nconv,
            const double *d_coef, double *out) {
  if (nconv < 0 || nconv > MAXV) return set_error(SBCI_EINVAL, "deflate: too many roots");
  RedBuf r;
  SBCI_TRY(red_buf(ctx, r));
  Ptrs p{};
  for (int i = 0; i < nconv; ++i) p.p[i] = xc[i];
  if (nconv <= 4)
    k_deflate<T, 4><<<grid_for(n), BS, 0, ctx->stream>>>(n, w, x, y, p, nconv, d_coef, r.part,
                                                         r.ticket, out);
  else
    k_deflate<T, MAXV><<<grid_for(n), BS, 0, ctx->stream>>>(n, w, x, y, p, nconv, d_coef, r.part,
                                                            r.ticket, out);
  k_reduce<<<1, BS, 0, ctx->stream>>>(r.part, grid_for(n), 3, out);
  SBCI_CHECK_LAUNCH();
  return SBCI_OK;
}

template <typename T>
int resid(sbci_ctx *ctx, int64_t n, const T *x, const T *X, const T *D, double E, double inv,
          double E0, double floor, const T *const *xc, int nconv, T *w, double *out) {
  if (nconv < 0 || nconv > MAXV) return set_error(SBCI_EINVAL, "resid: too many roots");
  RedBuf r;
  SBCI_TRY(red_buf(ctx, r));
  Ptrs p{};
  for (int i = 0; i < nconv; ++i) p.p[i] = xc[i];
  if (nconv <= 4)
    k_resid<T, 4><<<grid_for(n), BS, 0, ctx->stream>>>(n, x, X, D, E, inv, E0, floor, p, nconv, w,
                                                       r.part, r.ticket, out);
  else
    k_resid<T, MAXV><<<grid_for(n), BS, 0, ctx->stream>>>(n, x, X, D, E, inv, E0, floor, p, nconv,
                                                          w, r.part, r.ticket, out);
  k_reduce<<<1, BS, 0, ctx->stream>>>(r.part, grid_for(n), 1 + nconv, out);
  SBCI_CHECK_LAUNCH();
  return SBCI_OK;
}

template <typename T>
int dots_xyz(sbci_ctx *ctx, int64_t n, const T *x, const T *y, const T *z, const T *Z, double *out) {
  RedBuf r;
  SBCI_TRY(red_buf(ctx, r));
  k_dots_xyz<T><<<grid_for(n), BS, 0, ctx->stream>>>(n, x, y, z, Z, r.part, r.ticket, out);
  k_reduce<<<1, BS, 0, ctx->stream>>>(r.part, grid_for(n), 3, out);
  SBCI_CHECK_LAUNCH();
  return SBCI_OK;
}

int gram(sbci_ctx *ctx, int64_t n, const double *const *b, const double *const *h, int m,
         double *out) {
  if (m != 4 && m != 6) return set_error(SBCI_EINVAL, "gram: a basis of 4 or 6 vectors");
  RedBuf r;
  SBCI_TRY(red_buf(ctx, r));
  Ptrs pb{}, ph{};
  for (int i = 0; i < m; ++i) {
    pb.p[i] = b[i];
    ph.p[i] = h[i];
  }
  const int nq = m * (m + 1);
  if (m == 4)
    k_gram<4><<<grid_for(n), BS, 0, ctx->stream>>>(n, pb, ph, r.part, r.ticket, out);
  else
    k_gram<6><<<grid_for(n), BS, 0, ctx->stream>>>(n, pb, ph, r.part, r.ticket, out);
  k_reduce<<<1, BS, 0, ctx->stream>>>(r.part, grid_for(n), nq, out);
  SBCI_CHECK_LAUNCH();
  return SBCI_OK;
}

#define INST(T)                                                                                   \
  template int dots<T>(sbci_ctx *, int64_t, const T *, const T *const *, int, double *);         \
  template int lincomb<T>(sbci_ctx *, int64_t, T *, const T *const *, const double *, int, double); \
  template int update<T>(sbci_ctx *, int64_t, T *, T *, T *, T *, const T *, const T *, T *,      \
                         const T *, const T *const *, const UpdateArgs &, double *);              \
  template int deflate<T>(sbci_ctx *, int64_t, T *, const T *, const T *, const T *const *, int,  \
                          const double *, double *);                                              \
  template int dots_xyz<T>(sbci_ctx *, int64_t, const T *, const T *, const T *, const T *, double *); \
  template int resid<T>(sbci_ctx *, int64_t, const T *, const T *, const T *, double, double, double,  \
                        double, const T *const *, int, T *, double *);
INST(double)
INST(float)
#undef INST
template int convert<double, float>(sbci_ctx *, int64_t, double *, const float *, double);
template int convert<float, double>(sbci_ctx *, int64_t, float *, const double *, double);
template int convert<double, double>(sbci_ctx *, int64_t, double *, const double *, double);
template int convert<float, float>(sbci_ctx *, int64_t, float *, const float *, double);

}  // namespace sbci
