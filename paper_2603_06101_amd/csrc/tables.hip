// Strings, lexical addressing, single-excitation tables, same-spin
// Hamiltonian lists, pair-scatter tables and the diagonal D (one-time set-up
// of a context, all built on the device).
//
// Determinant basis of the paper's problem statement (Results, "SBCI1
// algorithm"); the determinant count C(N, n_alpha) * C(N, n_beta) is the one
// printed for every instance in Section S3.1.
//
// * strings: m-subsets of {0..N-1} as uint64 masks in ascending order; the
//   rank of a mask is sum_k C(o_k, k) over its occupied o_1 < ... < o_m
//   (combinatorial number system), so rank and order agree;
// * E_pq |I> = sign |I - q + p>, sign = (-1)^(occupied strictly between p, q);
// * same-spin list of string I: every J with a non-zero same-spin matrix
//   element <J| sum h_pq E_pq + 1/2 sum (pq|rs)(E_pq E_rs - d_qr E_ps) |I>
//   (within one spin), from the Slater-Condon rules: J = I (diagonal), the
//   m(N-m) singles and the C(m,2) C(N-m,2) doubles;
// * pair table: for string J and unordered orbital pair {k >= l}, the string
//   I' and sign with <I'| E_kl or E_lk |J> != 0 (at most one orientation is
//   non-zero), used to scatter the opposite-spin contraction.
#include "internal.h"

#include <cmath>
#include <cstring>

namespace sbci {

namespace {

__device__ __forceinline__ int64_t rank_of(uint64_t mask, const int64_t *__restrict__ binom) {
  int64_t r = 0;
  int k = 1;
  while (mask) {
    int o = __builtin_ctzll(mask);
    r += binom[o * 65 + k];
    ++k;
    mask &= mask - 1;
  }
  return r;
}

__device__ __forceinline__ int parity_between(uint64_t mask, int a, int b) {
  int lo = a < b ? a : b, hi = a < b ? b : a;
  if (hi - lo < 2) return 0;
  uint64_t m = ((1ull << hi) - 1) & ~((1ull << (lo + 1)) - 1);
  return __popcll(mask & m) & 1;
}

__global__ void k_strings(int norb, int m, int64_t ns, const int64_t *__restrict__ binom,
                          uint64_t *__restrict__ out) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= ns) return;
  int64_t r = i;
  uint64_t mask = 0;
  int o = norb - 1;
  for (int k = m; k >= 1; --k) {
    while (binom[o * 65 + k] > r) --o;
    mask |= 1ull << o;
    r -= binom[o * 65 + k];
    --o;
  }
  out[i] = mask;
}

__global__ void k_exc_table(int norb, int m, int64_t ns, int s, const uint64_t *__restrict__ str,
                            const int64_t *__restrict__ binom, Ent *__restrict__ tab) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= ns) return;
  const uint64_t mask = str[i];
  Ent *row = tab + i * s;
  int e = 0;
  for (int o = 0; o < norb; ++o) {
    if ((mask >> o) & 1) {
      Ent t;
      t.J = (int32_t)i;
      t.p = (uint8_t)o;
      t.q = (uint8_t)o;
      t.sign = 1;
      t.pad = 0;
      row[e++] = t;
    }
  }
  for (int q = 0; q < norb; ++q) {
    if (!((mask >> q) & 1)) continue;
    for (int p = 0; p < norb; ++p) {
      if ((mask >> p) & 1) continue;
      uint64_t nm = (mask & ~(1ull << q)) | (1ull << p);
      Ent t;
      t.J = (int32_t)rank_of(nm, binom);
      t.p = (uint8_t)p;
      t.q = (uint8_t)q;
      t.sign = parity_between(mask, p, q) ? -1 : 1;
      t.pad = 0;
      row[e++] = t;
    }
  }
}

__global__ void k_pair_table(int norb, int64_t ns, int64_t ns_pad, int npair, int npair_pad,
                             const uint64_t *__restrict__ str, const int64_t *__restrict__ binom,
                             uint32_t *__restrict__ pair) {
  int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int kl = blockIdx.y;
  if (j >= ns_pad || kl >= npair_pad) return;
  uint32_t code = kInvalid;
  if (kl < npair && j < ns) {
    int k = 0;
    while ((k + 1) * (k + 2) / 2 <= kl) ++k;
    int l = kl - k * (k + 1) / 2;
    const uint64_t mask = str[j];
    const int bk = (mask >> k) & 1, bl = (mask >> l) & 1;
    if (k == l) {
      if (bk) code = (uint32_t)j << 1;
    } else if (bk != bl) {
      // the occupied one of {k, l} moves to the empty one
      uint64_t nm = mask ^ (1ull << k) ^ (1ull << l);
      uint32_t tgt = (uint32_t)rank_of(nm, binom);
      code = (tgt << 1) | (uint32_t)parity_between(mask, k, l);
    }
  }
  pair[(int64_t)kl * ns_pad + j] = code;
}

// Pair-table quads: out[(u*4 + g) * ns_pad + J] = codes of rows
// u*16 + orow(g, r), r = 0..3, with orow = g + 4r (GP4R) or 4g + r.
template <bool GP4R>
__global__ void k_pair_quads(const uint32_t *__restrict__ pair, int64_t ns_pad, int ntiles,
                             uint4 *__restrict__ out) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)ntiles * 4 * ns_pad) return;
  const int64_t J = e % ns_pad, ug = e / ns_pad;
  const int g = (int)(ug & 3), u = (int)(ug >> 2);
  uint32_t c[4];
  for (int r = 0; r < 4; ++r) {
    const int64_t row = u * 16 + (GP4R ? g + 4 * r : 4 * g + r);
    c[r] = pair[row * ns_pad + J];
  }
  out[e] = make_uint4(c[0], c[1], c[2], c[3]);
}

// Orbital-grouped tables.  Strings holding orbital q correspond, in the same
// (ascending) order, to the (m-1)-subsets of the other N-1 orbitals: unrank
// j over C(N-1, m-1), lift the orbitals >= q by one and add q.
__global__ void k_colq(int norb, int m, int64_t nq, const int64_t *__restrict__ binom,
                       int32_t *__restrict__ colq) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (j >= nq) return;
  int64_t r = j;
  uint64_t mask = 1ull << q;
  int o = norb - 2;
  for (int k = m - 1; k >= 1; --k) {
    while (binom[o * 65 + k] > r) --o;
    mask |= 1ull << (o >= q ? o + 1 : o);
    r -= binom[o * 65 + k];
    --o;
  }
  colq[(int64_t)q * nq + j] = (int32_t)rank_of(mask, binom);
}

// out[((q * mt + u) * 4 + g) * nq_pad + j] = codes of E_pq colq[q][j] for
// p = u*16 + orow(g, r), r = 0..3 (orow = g + 4r if GP4R, else 4g + r).
template <bool GP4R>
__global__ void k_q_quads(int norb, int mt, int64_t nq, int64_t nq_pad,
                          const int32_t *__restrict__ colq, const uint64_t *__restrict__ str,
                          const int64_t *__restrict__ binom, uint4 *__restrict__ out) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int qug = blockIdx.y;  // (q * mt + u) * 4 + g
  if (j >= nq_pad) return;
  const int g = qug & 3, u = (qug >> 2) % mt, q = (qug >> 2) / mt;
  uint32_t c[4] = {kInvalid, kInvalid, kInvalid, kInvalid};
  if (j < nq) {
    const int64_t J = colq[(int64_t)q * nq + j];
    const uint64_t mask = str[J];
    for (int r = 0; r < 4; ++r) {
      const int p = u * 16 + (GP4R ? g + 4 * r : 4 * g + r);
      if (p >= norb) continue;
      if (p == q) {
        c[r] = (uint32_t)J << 1;
      } else if (!((mask >> p) & 1)) {
        const uint64_t nm = (mask & ~(1ull << q)) | (1ull << p);
        c[r] = ((uint32_t)rank_of(nm, binom) << 1) | (uint32_t)parity_between(mask, p, q);
      }
    }
  }
  out[(int64_t)qug * nq_pad + j] = make_uint4(c[0], c[1], c[2], c[3]);
}

// dst[f][i] = src[i][f] for an [ns][nf] list array
template <typename T>
__global__ void k_list_t(const T *__restrict__ src, T *__restrict__ dst, int64_t ns, int nf) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= ns * nf) return;
  const int64_t i = e / nf, f = e - i * nf;
  dst[f * ns + i] = src[e];
}

// Block-binned lists: per 64-row group (one wave, lane = row), the largest
// number of entries any row of the group has in each source block.
__global__ __launch_bounds__(64) void k_blk_count(const int32_t *__restrict__ fcol, int nf,
                                                  int64_t ns, int nblk, int rb,
                                                  int32_t *__restrict__ kmax) {
  __shared__ int cnt[kSameBlkMaxBlocks][64];
  const int lane = threadIdx.x;
  const int64_t g = blockIdx.x, I = g * 64 + lane;
  for (int b = 0; b < nblk; ++b) cnt[b][lane] = 0;
  if (I < ns)
    for (int e = 0; e < nf; ++e) cnt[fcol[I * nf + e] / rb][lane] += 1;
  __syncthreads();
  for (int b = lane; b < nblk; b += 64) {
    int m = 0;
    for (int l = 0; l < 64; ++l) m = max(m, cnt[b][l]);
    kmax[g * nblk + b] = m;
  }
}

// Fill the block-binned lists (entries in list order within each block),
// then pad every row's block segment to the group's length.
__global__ __launch_bounds__(64) void k_blk_fill(const int32_t *__restrict__ fcol,
                                                 const double *__restrict__ f64,
                                                 const float *__restrict__ f32, int nf, int64_t ns,
                                                 int nblk, int rb, const int32_t *__restrict__ boff,
                                                 uint16_t *__restrict__ bcol,
                                                 double *__restrict__ b64, float *__restrict__ b32) {
  __shared__ int cnt[kSameBlkMaxBlocks][64];
  const int lane = threadIdx.x;
  const int64_t g = blockIdx.x, I = g * 64 + lane;
  for (int b = 0; b < nblk; ++b) cnt[b][lane] = 0;
  if (I < ns)
    for (int e = 0; e < nf; ++e) {
      const int col = fcol[I * nf + e];
      const int b = col / rb;
      const int64_t slot = (int64_t)boff[g * nblk + b] + cnt[b][lane]++;
      bcol[slot * 64 + lane] = (uint16_t)(col - b * rb);
      b64[slot * 64 + lane] = f64[I * nf + e];
      b32[slot * 64 + lane] = f32[I * nf + e];
    }
  for (int b = 0; b < nblk; ++b)
    for (int64_t slot = (int64_t)boff[g * nblk + b] + cnt[b][lane]; slot < boff[g * nblk + b + 1];
         ++slot) {
      bcol[slot * 64 + lane] = 0;
      b64[slot * 64 + lane] = 0.0;
      b32[slot * 64 + lane] = 0.0f;
    }
}

__device__ __forceinline__ double G4(const double *__restrict__ g, int n, int p, int q, int r, int s) {
  return g[((p * n + q) * n + r) * n + s];
}

// Each row's same-spin list in ascending column order (one workgroup per
// row: bitonic sort of (column, entry) keys in LDS, values permuted along).
// Rows of neighbouring strings then reach their shared targets at the same
// list position, so the lanes of a wave, which own neighbouring rows, often
// read the same source row together in the LDS-staged products.  Measured
// at CAS(16,16) and CAS(14,14): 1-2 % off the same-spin kernels.  kp: nf
// rounded up to a power of two, at most kSortListMax.
constexpr int kSortListMax = 4096;

__global__ __launch_bounds__(256) void k_sort_flist(int nf, int kp, int32_t *__restrict__ fcol,
                                                    double *__restrict__ f64, float *__restrict__ f32) {
  extern __shared__ __align__(16) unsigned char smem[];
  uint64_t *key = reinterpret_cast<uint64_t *>(smem);   // [kp]
  double *v64 = reinterpret_cast<double *>(key + kp);    // [nf]
  float *v32 = reinterpret_cast<float *>(v64 + nf);      // [nf]
  const int64_t row = blockIdx.x;
  int32_t *col = fcol + row * nf;
  double *d = f64 + row * nf;
  float *f = f32 + row * nf;
  for (int e = threadIdx.x; e < kp; e += 256) {
    if (e < nf) {
      key[e] = ((uint64_t)(uint32_t)col[e] << 16) | (uint64_t)e;
      v64[e] = d[e];
      v32[e] = f[e];
    } else {
      key[e] = ~0ull;
    }
  }
  __syncthreads();
  for (int k = 2; k <= kp; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < kp; i += 256) {
        const int l = i ^ j;
        if (l > i) {
          const uint64_t a = key[i], b = key[l];
          const bool up = (i & k) == 0;
          if ((a > b) == up) {
            key[i] = b;
            key[l] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int e = threadIdx.x; e < nf; e += 256) {
    const uint64_t kk = key[e];
    const int src = (int)(kk & 0xffffu);
    col[e] = (int32_t)(kk >> 16);
    d[e] = v64[src];
    f[e] = v32[src];
  }
}

__global__ void k_flist(int norb, int m, int64_t ns, int nf, const uint64_t *__restrict__ str,
                        const int64_t *__restrict__ binom, const double *__restrict__ h,
                        const double *__restrict__ g, int32_t *__restrict__ fcol,
                        double *__restrict__ f64, float *__restrict__ f32,
                        double *__restrict__ fdiag) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= ns) return;
  const int n = norb;
  const uint64_t mask = str[i];
  int32_t *col = fcol + i * nf;
  double *val = f64 + i * nf;
  float *val32 = f32 + i * nf;
  int e = 0;
  // diagonal: sum_p h_pp + 1/2 sum_{p,q in I} [(pp|qq) - (pq|qp)]
  double d = 0.0;
  for (int p = 0; p < n; ++p) {
    if (!((mask >> p) & 1)) continue;
    d += h[p * n + p];
    for (int q = 0; q < n; ++q)
      if ((mask >> q) & 1) d += 0.5 * (G4(g, n, p, p, q, q) - G4(g, n, p, q, q, p));
  }
  fdiag[i] = d;
  col[e] = (int32_t)i;
  val[e] = d;
  val32[e] = (float)d;
  ++e;
  // singles q -> p: sign * [h_pq + sum_{r in I, r != q} ((pq|rr) - (pr|rq))]
  for (int q = 0; q < n; ++q) {
    if (!((mask >> q) & 1)) continue;
    for (int p = 0; p < n; ++p) {
      if ((mask >> p) & 1) continue;
      double v = h[p * n + q];
      for (int r = 0; r < n; ++r)
        if (r != q && ((mask >> r) & 1)) v += G4(g, n, p, q, r, r) - G4(g, n, p, r, r, q);
      if (parity_between(mask, p, q)) v = -v;
      uint64_t nm = (mask & ~(1ull << q)) | (1ull << p);
      col[e] = (int32_t)rank_of(nm, binom);
      val[e] = v;
      val32[e] = (float)v;
      ++e;
    }
  }
  // doubles (q1 < q2) -> (p1 < p2): sign * [(p1 q1|p2 q2) - (p1 q2|p2 q1)]
  for (int q1 = 0; q1 < n; ++q1) {
    if (!((mask >> q1) & 1)) continue;
    for (int q2 = q1 + 1; q2 < n; ++q2) {
      if (!((mask >> q2) & 1)) continue;
      for (int p1 = 0; p1 < n; ++p1) {
        if ((mask >> p1) & 1) continue;
        for (int p2 = p1 + 1; p2 < n; ++p2) {
          if ((mask >> p2) & 1) continue;
          double v = G4(g, n, p1, q1, p2, q2) - G4(g, n, p1, q2, p2, q1);
          uint64_t m1 = (mask & ~(1ull << q2)) | (1ull << p2);
          int neg = parity_between(mask, p2, q2) ^ parity_between(m1, p1, q1);
          uint64_t m2 = (m1 & ~(1ull << q1)) | (1ull << p1);
          col[e] = (int32_t)rank_of(m2, binom);
          val[e] = neg ? -v : v;
          val32[e] = (float)val[e];
          ++e;
        }
      }
    }
  }
}

// D[Ia, Ib] = fdiag_a[Ia] + fdiag_b[Ib] + sum_{p in Ia, q in Ib} (pp|qq)
__global__ void k_hdiag(int norb, int64_t nsa, int64_t nsb, const uint64_t *__restrict__ sa,
                        const uint64_t *__restrict__ sb, const double *__restrict__ fa,
                        const double *__restrict__ fb, const double *__restrict__ g,
                        double *__restrict__ D, float *__restrict__ D32) {
  __shared__ double J[64 * 64];
  const int n = norb;
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    int p = t / n, q = t % n;
    J[t] = G4(g, n, p, p, q, q);
  }
  __syncthreads();
  const int64_t ndet = nsa * nsb;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ndet;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ia = i / nsb, ib = i - ia * nsb;
    uint64_t ma = sa[ia];
    const uint64_t mb = sb[ib];
    double e = fa[ia] + fb[ib];
    while (ma) {
      int p = __builtin_ctzll(ma);
      ma &= ma - 1;
      uint64_t mm = mb;
      while (mm) {
        int q = __builtin_ctzll(mm);
        mm &= mm - 1;
        e += J[p * n + q];
      }
    }
    D[i] = e;
    D32[i] = (float)e;
  }
}

int64_t choose_host(int n, int k) {
  static int64_t t[65][65];
  static bool ready = false;
  if (!ready) {
    for (int i = 0; i <= 64; ++i) {
      t[i][0] = 1;
      for (int j = 1; j <= 64; ++j) t[i][j] = i == 0 ? 0 : t[i - 1][j - 1] + t[i - 1][j];
    }
    ready = true;
  }
  if (n < 0 || k < 0 || k > n || n > 64) return 0;
  return t[n][k];
}

int build_spin(sbci_ctx *ctx, SpinTables &T, int m) {
  const int n = ctx->norb;
  T.m = m;
  T.ns = choose_host(n, m);
  T.s = m * (n - m + 1);
  const int64_t nd = choose_host(m, 2) * choose_host(n - m, 2);
  T.nf = (int)(1 + (int64_t)m * (n - m) + nd);
  if (T.ns > INT32_MAX / 2) return set_error(SBCI_EINVAL, "string count exceeds int32 addressing");
  hipStream_t st = ctx->stream;
  SBCI_HIP(hipMalloc(&T.str, sizeof(uint64_t) * T.ns));
  SBCI_HIP(hipMalloc(&T.tab, sizeof(Ent) * T.ns * (T.s > 0 ? T.s : 1)));
  T.ns_pad = (T.ns + 15) / 16 * 16;
  SBCI_HIP(hipMalloc(&T.pair, sizeof(uint32_t) * T.ns_pad * ctx->npair_pad));
  SBCI_HIP(hipMalloc(&T.fcol, sizeof(int32_t) * T.ns * T.nf));
  SBCI_HIP(hipMalloc(&T.fval64, sizeof(double) * T.ns * T.nf));
  SBCI_HIP(hipMalloc(&T.fval32, sizeof(float) * T.ns * T.nf));
  SBCI_HIP(hipMalloc(&T.fdiag, sizeof(double) * T.ns));
  const int bs = 128;
  const unsigned gx = (unsigned)((T.ns + bs - 1) / bs);
  k_strings<<<gx, bs, 0, st>>>(n, m, T.ns, ctx->binom, T.str);
  SBCI_CHECK_LAUNCH();
  if (T.s > 0) {
    k_exc_table<<<gx, bs, 0, st>>>(n, m, T.ns, T.s, T.str, ctx->binom, T.tab);
    SBCI_CHECK_LAUNCH();
  }
  const unsigned gxp = (unsigned)((T.ns_pad + bs - 1) / bs);
  k_pair_table<<<dim3(gxp, ctx->npair_pad), bs, 0, st>>>(n, T.ns, T.ns_pad, ctx->npair,
                                                         ctx->npair_pad, T.str, ctx->binom, T.pair);
  SBCI_CHECK_LAUNCH();
  {
    const int ntiles = ctx->npair_pad / 16;
    const int64_t nq = (int64_t)ntiles * 4 * T.ns_pad;
    SBCI_HIP(hipMalloc(&T.quad_r, sizeof(uint4) * nq));
    SBCI_HIP(hipMalloc(&T.quad_s, sizeof(uint4) * nq));
    const unsigned gq = (unsigned)((nq + 255) / 256);
    k_pair_quads<false><<<gq, 256, 0, st>>>(T.pair, T.ns_pad, ntiles, T.quad_r);
    k_pair_quads<true><<<gq, 256, 0, st>>>(T.pair, T.ns_pad, ntiles, T.quad_s);
    SBCI_CHECK_LAUNCH();
  }
  if (m > 0) {
    T.nq = choose_host(n - 1, m - 1);
    T.nq_pad = (T.nq + 15) / 16 * 16;
    T.mt = (n + 15) / 16;
    SBCI_HIP(hipMalloc(&T.colq, sizeof(int32_t) * T.nq * n));
    const int64_t nqq = (int64_t)n * T.mt * 4 * T.nq_pad;
    SBCI_HIP(hipMalloc(&T.qquad_r, sizeof(uint4) * nqq));
    SBCI_HIP(hipMalloc(&T.qquad_s, sizeof(uint4) * nqq));
    k_colq<<<dim3((unsigned)((T.nq + bs - 1) / bs), n), bs, 0, st>>>(n, m, T.nq, ctx->binom, T.colq);
    SBCI_CHECK_LAUNCH();
    const dim3 gq((unsigned)((T.nq_pad + bs - 1) / bs), (unsigned)(n * T.mt * 4));
    k_q_quads<false><<<gq, bs, 0, st>>>(n, T.mt, T.nq, T.nq_pad, T.colq, T.str, ctx->binom,
                                        T.qquad_r);
    k_q_quads<true><<<gq, bs, 0, st>>>(n, T.mt, T.nq, T.nq_pad, T.colq, T.str, ctx->binom,
                                       T.qquad_s);
    SBCI_CHECK_LAUNCH();
  }
  const int fbs = 64;  // heavy per-thread loops: small blocks
  k_flist<<<(unsigned)((T.ns + fbs - 1) / fbs), fbs, 0, st>>>(n, m, T.ns, T.nf, T.str, ctx->binom,
                                                              ctx->h1, ctx->eri, T.fcol, T.fval64,
                                                              T.fval32, T.fdiag);
  SBCI_CHECK_LAUNCH();
  {
    int kp = 1;
    while (kp < T.nf) kp <<= 1;
    if (T.nf > 1 && kp <= kSortListMax) {
      const size_t lds = (size_t)kp * 8 + (size_t)T.nf * 12;
      static bool attr = false;
      if (!attr) {
        SBCI_HIP(hipFuncSetAttribute((const void *)k_sort_flist,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024));
        attr = true;
      }
      k_sort_flist<<<(unsigned)T.ns, 256, lds, st>>>(T.nf, kp, T.fcol, T.fval64, T.fval32);
      SBCI_CHECK_LAUNCH();
    }
  }
  if (T.ns >= kSameLdsMinRows && T.ns <= kSameLdsMaxRows) {
    const int64_t ne = T.ns * (int64_t)T.nf;
    SBCI_HIP(hipMalloc(&T.fcolT, sizeof(int32_t) * ne));
    SBCI_HIP(hipMalloc(&T.fvalT64, sizeof(double) * ne));
    SBCI_HIP(hipMalloc(&T.fvalT32, sizeof(float) * ne));
    const unsigned g = (unsigned)((ne + 255) / 256);
    k_list_t<int32_t><<<g, 256, 0, st>>>(T.fcol, T.fcolT, T.ns, T.nf);
    k_list_t<double><<<g, 256, 0, st>>>(T.fval64, T.fvalT64, T.ns, T.nf);
    k_list_t<float><<<g, 256, 0, st>>>(T.fval32, T.fvalT32, T.ns, T.nf);
    SBCI_CHECK_LAUNCH();
  }
  return SBCI_OK;
}

}  // namespace

int build_blk_lists(sbci_ctx *ctx, SpinTables &T) {
  if (T.bcol) return SBCI_OK;
  const int rb = kSameBlkRows;
  const int nblk = (int)((T.ns + rb - 1) / rb);
  if (nblk > kSameBlkMaxBlocks || T.nf < 1)
    return set_error(SBCI_EINVAL, "same-spin sigma: too many strings for the blocked LDS form");
  const int64_t ngrp = (T.ns + 63) / 64;
  hipStream_t st = ctx->stream;
  int32_t *kmax = nullptr;
  SBCI_HIP(hipMalloc(&kmax, sizeof(int32_t) * ngrp * nblk));
  struct Free {
    void *p;
    ~Free() { hipFree(p); }
  } guard{kmax};
  k_blk_count<<<(unsigned)ngrp, 64, 0, st>>>(T.fcol, T.nf, T.ns, nblk, rb, kmax);
  SBCI_CHECK_LAUNCH();
  std::vector<int32_t> k((size_t)(ngrp * nblk)), off((size_t)(ngrp * nblk + 1));
  SBCI_HIP(hipMemcpyAsync(k.data(), kmax, sizeof(int32_t) * k.size(), hipMemcpyDeviceToHost, st));
  SBCI_HIP(hipStreamSynchronize(st));
  int64_t acc = 0;
  for (size_t i = 0; i < k.size(); ++i) {
    off[i] = (int32_t)acc;
    acc += k[i];
  }
  off[k.size()] = (int32_t)acc;
  if (acc >= ((int64_t)1 << 31) / 64)
    return set_error(SBCI_EINVAL, "same-spin sigma: blocked lists too large");
  const int64_t slots = acc > 0 ? acc : 1;
  SBCI_HIP(hipMalloc(&T.boff, sizeof(int32_t) * off.size()));
  SBCI_HIP(hipMalloc(&T.bcol, sizeof(uint16_t) * slots * 64));
  SBCI_HIP(hipMalloc(&T.bval64, sizeof(double) * slots * 64));
  SBCI_HIP(hipMalloc(&T.bval32, sizeof(float) * slots * 64));
  SBCI_HIP(hipMemcpyAsync(T.boff, off.data(), sizeof(int32_t) * off.size(), hipMemcpyHostToDevice, st));
  k_blk_fill<<<(unsigned)ngrp, 64, 0, st>>>(T.fcol, T.fval64, T.fval32, T.nf, T.ns, nblk, rb, T.boff,
                                           T.bcol, T.bval64, T.bval32);
  SBCI_CHECK_LAUNCH();
  SBCI_HIP(hipStreamSynchronize(st));  // off[] and kmax stay valid until here
  T.nblk = nblk;
  T.ngrp = ngrp;
  return SBCI_OK;
}

namespace {

void free_spin(SpinTables &T) {
  if (T.shared) {
    T = SpinTables();
    return;
  }
  hipFree(T.str);
  hipFree(T.tab);
  hipFree(T.pair);
  hipFree(T.fcol);
  hipFree(T.fval64);
  hipFree(T.fval32);
  hipFree(T.fdiag);
  hipFree(T.quad_r);
  hipFree(T.quad_s);
  hipFree(T.colq);
  hipFree(T.hd64);
  hipFree(T.hd32);
  hipFree(T.hdbf);
  hipFree(T.hdd32);
  hipFree(T.qquad_r);
  hipFree(T.qquad_s);
  hipFree(T.fcolT);
  hipFree(T.fvalT64);
  hipFree(T.fvalT32);
  hipFree(T.boff);
  hipFree(T.bcol);
  hipFree(T.bval64);
  hipFree(T.bval32);
  T = SpinTables();
}

}  // namespace

int build_tables(sbci_ctx *ctx, const double *h1, const double *eri) {
  const int n = ctx->norb;
  ctx->npair = n * (n + 1) / 2;
  ctx->npair_pad = 16 * ((ctx->npair + 15) / 16 + 9);
  hipStream_t st = ctx->stream;
  // binomial table [65][65]
  std::vector<int64_t> binom(65 * 65);
  for (int i = 0; i <= 64; ++i)
    for (int k = 0; k <= 64; ++k) binom[i * 65 + k] = choose_host(i, k);
  SBCI_HIP(hipMalloc(&ctx->binom, sizeof(int64_t) * 65 * 65));
  SBCI_HIP(hipMemcpyAsync(ctx->binom, binom.data(), sizeof(int64_t) * 65 * 65,
                          hipMemcpyHostToDevice, st));
  const size_t n4 = (size_t)n * n * n * n;
  SBCI_HIP(hipMalloc(&ctx->h1, sizeof(double) * n * n));
  SBCI_HIP(hipMalloc(&ctx->eri, sizeof(double) * n4));
  SBCI_HIP(hipMemcpyAsync(ctx->h1, h1, sizeof(double) * n * n, hipMemcpyHostToDevice, st));
  SBCI_HIP(hipMemcpyAsync(ctx->eri, eri, sizeof(double) * n4, hipMemcpyHostToDevice, st));
  // packed-pair ERI matrix W[kl][k'l'] = (kl|k'l'), k >= l
  const int np = ctx->npair;
  std::vector<double> W((size_t)np * np);
  std::vector<float> W32((size_t)np * np);
  std::vector<__hip_bfloat16> Wbf((size_t)np * np);
  std::vector<int> pk(np), pl(np);
  for (int k = 0, kl = 0; k < n; ++k)
    for (int l = 0; l <= k; ++l, ++kl) pk[kl] = k, pl[kl] = l;
  for (int a = 0; a < np; ++a)
    for (int b = 0; b < np; ++b) {
      double v = eri[((size_t)(pk[a] * n + pl[a]) * n + pk[b]) * n + pl[b]];
      W[(size_t)a * np + b] = v;
      W32[(size_t)a * np + b] = (float)v;
      Wbf[(size_t)a * np + b] = __float2bfloat16((float)v);
    }
  SBCI_HIP(hipMalloc(&ctx->W64, sizeof(double) * np * np));
  SBCI_HIP(hipMalloc(&ctx->W32, sizeof(float) * np * np));
  SBCI_HIP(hipMalloc(&ctx->Wbf, sizeof(__hip_bfloat16) * np * np));
  SBCI_HIP(hipMemcpyAsync(ctx->W64, W.data(), sizeof(double) * np * np, hipMemcpyHostToDevice, st));
  SBCI_HIP(hipMemcpyAsync(ctx->W32, W32.data(), sizeof(float) * np * np, hipMemcpyHostToDevice, st));
  SBCI_HIP(hipMemcpyAsync(ctx->Wbf, Wbf.data(), sizeof(__hip_bfloat16) * np * np,
                          hipMemcpyHostToDevice, st));
  {
    double rmax = 0;
    for (int a = 0; a < np; ++a) {
      double r = 0;
      for (int b = 0; b < np; ++b) r += std::fabs(W[(size_t)a * np + b]);
      rmax = std::fmax(rmax, r);
    }
    const int mb = ctx->nb;
    ctx->opp_wbound = (double)(mb * (n - mb + 1)) * rmax;
  }
  SBCI_TRY(build_spin(ctx, ctx->A, ctx->na));
  if (ctx->nb == ctx->na) {
    ctx->B = ctx->A;
    ctx->B.shared = true;
  } else {
    SBCI_TRY(build_spin(ctx, ctx->B, ctx->nb));
  }
  ctx->ndet = ctx->A.ns * ctx->B.ns;
  SBCI_HIP(hipMalloc(&ctx->hdiag, sizeof(double) * ctx->ndet));
  SBCI_HIP(hipMalloc(&ctx->hdiag32, sizeof(float) * ctx->ndet));
  int64_t blocks = (ctx->ndet + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  k_hdiag<<<(unsigned)blocks, 256, 0, st>>>(n, ctx->A.ns, ctx->B.ns, ctx->A.str, ctx->B.str,
                                            ctx->A.fdiag, ctx->B.fdiag, ctx->eri, ctx->hdiag,
                                            ctx->hdiag32);
  SBCI_CHECK_LAUNCH();
  SBCI_HIP(hipStreamSynchronize(st));  // host vectors above must outlive the copies
  return SBCI_OK;
}

void free_tables(sbci_ctx *ctx) {
  free_spin(ctx->B);
  free_spin(ctx->A);
  hipFree(ctx->binom);
  hipFree(ctx->h1);
  hipFree(ctx->eri);
  hipFree(ctx->W64);
  hipFree(ctx->W32);
  hipFree(ctx->Wbf);
  hipFree(ctx->hdiag);
  hipFree(ctx->hdiag32);
  ctx->binom = nullptr;
  ctx->h1 = ctx->eri = ctx->W64 = ctx->hdiag = nullptr;
  ctx->W32 = ctx->hdiag32 = nullptr;
  ctx->Wbf = nullptr;
}

}  // namespace sbci
