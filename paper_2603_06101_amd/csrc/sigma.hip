// sigma = H c over alpha/beta strings on gfx950.
//
// The Hamiltonian of the paper's problem statement splits exactly into
//   H = H_alpha + H_beta + sum_{kl, k'l'} (kl|k'l') E^alpha_kl E^beta_k'l'
// where H_s = sum h_pq E^s_pq + 1/2 sum (pq|rs)(E^s_pq E^s_rs - d_qr E^s_ps)
// acts on one spin only.  The sigma build is the "matrix-product
// construction" whose cost dominates every SBCI and Davidson step
// (Introduction; the one sigma per SBCI step is Eq. S32).
//
// Kernels (C is row-major [Ia][Ib]):
//   k_same      sigma[r][c] (+)= sum_e F[r][e] * src[col(r,e)][c]: the
//               alpha part on C directly and the beta part on C^T (then
//               added back transposed).  List entries are wave-uniform
//               (scalar loads); row segments are coalesced vector loads.
//   k_opp       the opposite-spin part as a D * (pq|rs) * E contraction on
//               MFMA, one output row Ia per workgroup: the s alpha
//               excitations of Ia gather s rows of C (signed), a dense
//               (npair x s) x (s x 16) MFMA tile contraction with the ERI
//               pair matrix produces M[kl][J], and each M[kl][J] is
//               scattered through the beta pair table into an LDS copy of
//               sigma's row Ia (LDS atomics), written back once.
//   k_transpose / k_add_t   tiled transposes through LDS.
#include "internal.h"

namespace sbci {

namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

constexpr int TT = 32;  // transpose tile

template <typename T>
__global__ void k_transpose(const T *__restrict__ src, T *__restrict__ dst, int64_t R, int64_t C) {
  __shared__ T tile[TT][TT + 1];
  const int64_t vo = (int64_t)blockIdx.z * R * C;
  const int64_t r0 = (int64_t)blockIdx.y * TT, c0 = (int64_t)blockIdx.x * TT;
  for (int i = threadIdx.y; i < TT; i += blockDim.y) {
    int64_t r = r0 + i, c = c0 + threadIdx.x;
    if (r < R && c < C) tile[i][threadIdx.x] = src[vo + r * C + c];
  }
  __syncthreads();
  for (int i = threadIdx.y; i < TT; i += blockDim.y) {
    int64_t c = c0 + i, r = r0 + threadIdx.x;
    if (r < R && c < C) dst[vo + c * R + r] = tile[threadIdx.x][i];
  }
}

// dst[c][r] += src[r][c]  (src is [R][C], dst is [C][R])
template <typename T>
__global__ void k_add_t(const T *__restrict__ src, T *__restrict__ dst, int64_t R, int64_t C) {
  __shared__ T tile[TT][TT + 1];
  const int64_t vo = (int64_t)blockIdx.z * R * C;
  const int64_t r0 = (int64_t)blockIdx.y * TT, c0 = (int64_t)blockIdx.x * TT;
  for (int i = threadIdx.y; i < TT; i += blockDim.y) {
    int64_t r = r0 + i, c = c0 + threadIdx.x;
    if (r < R && c < C) tile[i][threadIdx.x] = src[vo + r * C + c];
  }
  __syncthreads();
  for (int i = threadIdx.y; i < TT; i += blockDim.y) {
    int64_t c = c0 + i, r = r0 + threadIdx.x;
    if (r < R && c < C) dst[vo + c * R + r] += tile[threadIdx.x][i];
  }
}

// One wave per list row r, 64 consecutive columns per wave.
template <typename T, typename V, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_same(
    const int32_t *__restrict__ fcol, const V *__restrict__ fval, int nf, int64_t R, int64_t C,
    const T *__restrict__ src, T *__restrict__ dst, int accumulate) {
  const int lane = threadIdx.x & 63;
  const int64_t r = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * WAVES + (threadIdx.x >> 6)));
  if (r >= R) return;
  const int64_t c = (int64_t)blockIdx.y * 64 + lane;
  const bool ok = c < C;
  const int64_t cc = ok ? c : C - 1;
  const int64_t vo = (int64_t)blockIdx.z * R * C;
  const T *__restrict__ s = src + vo + cc;
  const int32_t *__restrict__ col = fcol + r * nf;
  const V *__restrict__ val = fval + r * nf;
  T acc0 = 0, acc1 = 0;
  int e = 0;
  for (; e + 8 <= nf; e += 8) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = s[(int64_t)col[e + u] * C];
#pragma unroll
    for (int u = 0; u < 8; u += 2) {
      acc0 += (T)val[e + u] * v[u];
      acc1 += (T)val[e + u + 1] * v[u + 1];
    }
  }
  for (; e < nf; ++e) acc0 += (T)val[e] * s[(int64_t)col[e] * C];
  if (ok) {
    T *d = dst + vo + r * C + c;
    *d = accumulate ? *d + (acc0 + acc1) : (acc0 + acc1);
  }
}

// MFMA flavours of the opposite-spin contraction.
struct MF64 {
  using A = double;      // LDS element of the A (ERI) and B (gathered C) tiles
  using Acc = double;    // LDS accumulation of sigma's row
  using Frag = double;
  using Out = d4_t;
  static constexpr int KSTEP = 4;   // K per MFMA
  static constexpr int KPL = 1;     // K elements per lane per MFMA
  // output row held by lane group g, register r (measured on gfx950: the
  // f64 16x16x4 result interleaves rows across lane groups)
  __device__ static int orow(int g, int r) { return g + 4 * r; }
  template <typename T> __device__ static A cvt(T x) { return (A)x; }
  __device__ static Out mma(Frag a, Frag b, Out c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
struct MF32 {
  using A = float;
  using Acc = float;
  using Frag = float;
  using Out = f4_t;
  static constexpr int KSTEP = 4;
  static constexpr int KPL = 1;
  __device__ static int orow(int g, int r) { return 4 * g + r; }
  template <typename T> __device__ static A cvt(T x) { return (A)x; }
  __device__ static Out mma(Frag a, Frag b, Out c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
struct MBF16 {
  using A = __bf16;
  using Acc = float;
  using Frag = bf8_t;
  using Out = f4_t;
  static constexpr int KSTEP = 32;
  static constexpr int KPL = 8;
  __device__ static int orow(int g, int r) { return 4 * g + r; }
  template <typename T> __device__ static A cvt(T x) { return (__bf16)(float)x; }
  __device__ static Out mma(Frag a, Frag b, Out c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

__device__ __forceinline__ int pair_index(int p, int q) {
  int k = p > q ? p : q, l = p > q ? q : p;
  return k * (k + 1) / 2 + l;
}

// LDS layout (dynamic): acc[nsb] | Ws[MROWS][KW + PAD] | Rt[16][KW + PAD] | eJ[s] | eW[s]
// KW = kc_steps * KSTEP (K columns in one chunk), MROWS = Mt * 16.
template <typename M, typename T, int MTW>
__global__ __launch_bounds__(256) void k_opp(
    int64_t nsa, int64_t nsb, int s, int npair, int Mt, int kc_steps,
    const float *__restrict__ Wf, const double *__restrict__ Wd, const Ent *__restrict__ taba,
    const int32_t *__restrict__ pairb, const T *__restrict__ c, T *__restrict__ sigma) {
  using A = typename M::A;
  using Acc = typename M::Acc;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t ia = blockIdx.x;
  const int64_t vo = (int64_t)blockIdx.y * nsa * nsb;
  const int KW = kc_steps * M::KSTEP;
  const int LDW = KW + (M::KPL == 1 ? 1 : 8);  // padded row stride (elements)
  const int MROWS = Mt * 16;
  Acc *acc = reinterpret_cast<Acc *>(smem);
  size_t off = ((size_t)nsb * sizeof(Acc) + 15) & ~(size_t)15;
  A *Ws = reinterpret_cast<A *>(smem + off);
  off += (((size_t)MROWS * LDW * sizeof(A)) + 15) & ~(size_t)15;
  A *Rt = reinterpret_cast<A *>(smem + off);
  off += (((size_t)16 * LDW * sizeof(A)) + 15) & ~(size_t)15;
  int32_t *eJ = reinterpret_cast<int32_t *>(smem + off);
  off += (size_t)s * sizeof(int32_t);
  int32_t *eW = reinterpret_cast<int32_t *>(smem + off);  // pair index, sign in bit 31

  for (int e = tid; e < s; e += 256) {
    Ent t = taba[ia * s + e];
    eJ[e] = t.J;
    int kl = pair_index(t.p, t.q);
    eW[e] = t.sign < 0 ? (kl | (int32_t)0x80000000) : kl;
  }
  for (int64_t j = tid; j < nsb; j += 256) acc[j] = (Acc)0;
  __syncthreads();

  const T *__restrict__ cv = c + vo;
  const int nkc = (s + KW - 1) / KW;
  const int64_t njt = (nsb + 15) / 16;
  const int g = lane >> 4;   // lane group 0..3
  const int li = lane & 15;

  for (int kc = 0; kc < nkc; ++kc) {
    const int e0 = kc * KW;
    // A tile: Ws[row][k] = sign_e * (row | kl_e) for e = e0 + k
    for (int idx = tid; idx < MROWS * KW; idx += 256) {
      int row = idx / KW, k = idx - row * KW;
      int e = e0 + k;
      A v = M::cvt(0.0f);
      if (e < s && row < npair) {
        int w = eW[e];
        int kl = w & 0x7fffffff;
        double x = Wd ? Wd[(int64_t)row * npair + kl] : (double)Wf[(int64_t)row * npair + kl];
        v = M::cvt(w < 0 ? -x : x);
      }
      Ws[row * LDW + k] = v;
    }
    for (int64_t jt = 0; jt < njt; ++jt) {
      const int64_t j0 = jt * 16;
      __syncthreads();  // Ws ready / previous Rt consumed
      // B tile (transposed): Rt[j][k] = C[J_e][j0 + j]
      for (int idx = tid; idx < 16 * KW; idx += 256) {
        int k = idx >> 4, j = idx & 15;
        int e = e0 + k;
        A v = M::cvt(0.0f);
        if (e < s && j0 + j < nsb) v = M::cvt(cv[(int64_t)eJ[e] * nsb + j0 + j]);
        Rt[j * LDW + k] = v;
      }
      __syncthreads();
      for (int mb = 0; mb < Mt; mb += 4 * MTW) {
        typename M::Out out[MTW];
#pragma unroll
        for (int u = 0; u < MTW; ++u)
#pragma unroll
          for (int r = 0; r < 4; ++r) out[u][r] = 0;
        for (int ks = 0; ks < kc_steps; ++ks) {
          const int kb = ks * M::KSTEP + g * M::KPL;
          typename M::Frag bf;
          typename M::Frag af[MTW];
          if constexpr (M::KPL == 1) {
            bf = Rt[li * LDW + kb];
#pragma unroll
            for (int u = 0; u < MTW; ++u) {
              int mt = mb + wave + 4 * u;
              af[u] = mt < Mt ? Ws[(mt * 16 + li) * LDW + kb] : (A)0;
            }
          } else {
            bf = *reinterpret_cast<const bf8_t *>(&Rt[li * LDW + kb]);
#pragma unroll
            for (int u = 0; u < MTW; ++u) {
              int mt = mb + wave + 4 * u;
              int mrow = mt < Mt ? mt * 16 + li : 0;
              af[u] = *reinterpret_cast<const bf8_t *>(&Ws[mrow * LDW + kb]);
            }
          }
#pragma unroll
          for (int u = 0; u < MTW; ++u) out[u] = M::mma(af[u], bf, out[u]);
        }
        // scatter: out[u][r] = M[row = mt*16 + orow(g, r)][J = j0 + li]
        const int64_t J = j0 + li;
#pragma unroll
        for (int u = 0; u < MTW; ++u) {
          int mt = mb + wave + 4 * u;
          if (mt >= Mt || J >= nsb) continue;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            int row = mt * 16 + M::orow(g, r);
            if (row >= npair) continue;
            int32_t code = pairb[(int64_t)row * nsb + J];
            if (code == kInvalid) continue;
            Acc v = (Acc)out[u][r];
            if (code < 0) {
              code = ~code;
              v = -v;
            }
            atomicAdd(&acc[code], v);
          }
        }
      }
    }
    __syncthreads();  // all waves done with Ws before the next chunk overwrites it
  }
  __syncthreads();
  T *__restrict__ sv = sigma + vo + ia * nsb;
  for (int64_t j = tid; j < nsb; j += 256) sv[j] += (T)acc[j];
}

template <typename M, typename T>
int launch_opp(sbci_ctx *ctx, const T *c, T *out, int nvec) {
  const SpinTables &A = ctx->A, &B = ctx->B;
  if (A.s == 0 || B.m == 0) return SBCI_OK;
  const int npair = ctx->npair;
  const int Mt = (npair + 15) / 16;
  const int MROWS = Mt * 16;
  const int ksteps_total = (A.s + M::KSTEP - 1) / M::KSTEP;
  const size_t lds_cap = 160 * 1024;
  const size_t acc_b = ((size_t)B.ns * sizeof(typename M::Acc) + 15) & ~(size_t)15;
  const size_t ent_b = (size_t)A.s * 8;
  int kc = ksteps_total;
  auto need = [&](int k) {
    int KW = k * M::KSTEP, LDW = KW + (M::KPL == 1 ? 1 : 8);
    size_t ws = (((size_t)MROWS * LDW * sizeof(typename M::A)) + 15) & ~(size_t)15;
    size_t rt = (((size_t)16 * LDW * sizeof(typename M::A)) + 15) & ~(size_t)15;
    return acc_b + ws + rt + ent_b;
  };
  while (kc > 1 && need(kc) > lds_cap) --kc;
  if (need(kc) > lds_cap)
    return set_error(SBCI_EINVAL, "opposite-spin sigma: beta string count too large for LDS");
  const size_t lds = need(kc);
  const float *Wf = nullptr;
  const double *Wd = nullptr;
  if constexpr (std::is_same<typename M::A, double>::value) Wd = ctx->W64; else Wf = ctx->W32;
  dim3 grid((unsigned)A.ns, (unsigned)nvec);
  const int mtw_need = (Mt + 3) / 4;
  if (mtw_need <= 1) {
    k_opp<M, T, 1><<<grid, 256, lds, ctx->stream>>>(A.ns, B.ns, A.s, npair, Mt, kc, Wf, Wd, A.tab,
                                                    B.pair, c, out);
  } else if (mtw_need == 2) {
    k_opp<M, T, 2><<<grid, 256, lds, ctx->stream>>>(A.ns, B.ns, A.s, npair, Mt, kc, Wf, Wd, A.tab,
                                                    B.pair, c, out);
  } else {
    k_opp<M, T, 3><<<grid, 256, lds, ctx->stream>>>(A.ns, B.ns, A.s, npair, Mt, kc, Wf, Wd, A.tab,
                                                    B.pair, c, out);
  }
  SBCI_CHECK_LAUNCH();
  return SBCI_OK;
}

template <typename T, typename V>
int launch_same(sbci_ctx *ctx, const SpinTables &S, const V *fval, int64_t R, int64_t C,
                const T *src, T *dst, int nvec, int accumulate) {
  constexpr int WAVES = 4;
  dim3 grid((unsigned)((R + WAVES - 1) / WAVES), (unsigned)((C + 63) / 64), (unsigned)nvec);
  k_same<T, V, WAVES><<<grid, 64 * WAVES, 0, ctx->stream>>>(S.fcol, fval, S.nf, R, C, src, dst,
                                                           accumulate);
  SBCI_CHECK_LAUNCH();
  return SBCI_OK;
}

template <typename T>
int launch_transpose(sbci_ctx *ctx, const T *src, T *dst, int64_t R, int64_t C, int nvec, bool add) {
  dim3 grid((unsigned)((C + TT - 1) / TT), (unsigned)((R + TT - 1) / TT), (unsigned)nvec);
  dim3 block(TT, 8);
  if (add)
    k_add_t<T><<<grid, block, 0, ctx->stream>>>(src, dst, R, C);
  else
    k_transpose<T><<<grid, block, 0, ctx->stream>>>(src, dst, R, C);
  SBCI_CHECK_LAUNCH();
  return SBCI_OK;
}

template <typename T, typename M>
int sigma_t(sbci_ctx *ctx, const T *c, T *out, int nvec) {
  const SpinTables &A = ctx->A, &B = ctx->B;
  const int64_t na = A.ns, nb = B.ns;
  const size_t vbytes = sizeof(T) * (size_t)ctx->ndet * nvec;
  SBCI_TRY(ensure(ctx->ws_t, vbytes));
  SBCI_TRY(ensure(ctx->ws_s, vbytes));
  T *ct = static_cast<T *>(ctx->ws_t.ptr);
  T *st = static_cast<T *>(ctx->ws_s.ptr);
  const bool dbl = std::is_same<T, double>::value;
  // alpha part (plain write), then opposite-spin (accumulate)
  if (dbl)
    SBCI_TRY((launch_same<T, double>(ctx, A, A.fval64, na, nb, c, out, nvec, 0)));
  else
    SBCI_TRY((launch_same<T, float>(ctx, A, A.fval32, na, nb, c, out, nvec, 0)));
  SBCI_TRY((launch_opp<M, T>(ctx, c, out, nvec)));
  // beta part on C^T, added back transposed
  SBCI_TRY(launch_transpose<T>(ctx, c, ct, na, nb, nvec, false));
  if (dbl)
    SBCI_TRY((launch_same<T, double>(ctx, B, B.fval64, nb, na, ct, st, nvec, 0)));
  else
    SBCI_TRY((launch_same<T, float>(ctx, B, B.fval32, nb, na, ct, st, nvec, 0)));
  SBCI_TRY(launch_transpose<T>(ctx, st, out, nb, na, nvec, true));
  return SBCI_OK;
}

}  // namespace

int sigma(sbci_ctx *ctx, const void *c, void *out, int nvec, int mode) {
  switch (mode) {
    case SBCI_F64:
      return sigma_t<double, MF64>(ctx, static_cast<const double *>(c), static_cast<double *>(out),
                                   nvec);
    case SBCI_F32:
      return sigma_t<float, MF32>(ctx, static_cast<const float *>(c), static_cast<float *>(out),
                                  nvec);
    case SBCI_BF16:
      return sigma_t<float, MBF16>(ctx, static_cast<const float *>(c), static_cast<float *>(out),
                                   nvec);
    default:
      return set_error(SBCI_EINVAL, "unknown sigma dtype");
  }
}

}  // namespace sbci
