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
#include "mfma.h"

#include <mutex>

namespace sbci {

namespace {


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

// Dense same-spin product, the form for dilute spaces where a spin's
// same-spin operator is a sizeable fraction dense (about 19 % at
// CAS(6e,45o)) and its lists are too long to stream from L2:
//   out (+)= A B      A row-major [Mr][K], B row-major [K][N], out [Mr][N]
// with A = H_alpha (dense), B = C for the alpha part and A = C, B = H_beta
// for the beta part (both are plain row-major products, so no transposes).
// WM x WN waves per (64 WM) x (64 WN) output tile; K panels of 16 pass
// through registers into double-buffered LDS; each wave owns a 64 x 64 block
// of 4 x 4 MFMA tiles (FP64 16x16x4 or FP32 16x16x4).  Tiles are dealt to
// the 8 XCDs in contiguous ranges, row-panel-major, so the workgroups of one
// XCD share A's row panel in L2.  blockIdx.y selects the vector (strides sA,
// sB, sC; 0 for the shared operator).
template <typename M, typename T, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void k_gemm(int64_t Mr, int64_t N, int64_t K,
                                              const T *__restrict__ A, int64_t lda, int64_t sA,
                                              const T *__restrict__ B, int64_t ldb, int64_t sB,
                                              T *__restrict__ out, int64_t ldc, int64_t sC,
                                              int accumulate, int64_t tiles_n, int64_t per_xcd,
                                              int64_t total) {
  constexpr int BM = 64 * WM, BN = 64 * WN, BK = 16, NT = 64 * WM * WN;
  constexpr int LDA = BK + 1, LDB = BN + 4;
  // staging: each thread moves AE consecutive k of one A row and BE
  // consecutive columns of one B row per panel
  constexpr int AE = BM * BK / NT, BE = BK * BN / NT;
  static_assert(AE >= 1 && BE >= 1 && BK % AE == 0 && BN % BE == 0, "staging layout");
  __shared__ T As[2][BM * LDA];
  __shared__ T Bs[2][BK * LDB];
  const int64_t b = blockIdx.x;
  const int64_t w = (b & 7) * per_xcd + (b >> 3);
  if (w >= total) return;
  const int64_t tm = w / tiles_n, tn = w - tm * tiles_n;
  const int64_t r0 = tm * BM, c0 = tn * BN;
  const int64_t v = blockIdx.y;
  A += v * sA;
  B += v * sB;
  out += v * sC;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int wm = (wave / WN) * 64, wn = (wave % WN) * 64;
  const int ar = tid / (BK / AE), ak = (tid % (BK / AE)) * AE;
  const int bkr = tid / (BN / BE), bc = (tid % (BN / BE)) * BE;
  T ra[AE], rb[BE];
  auto load = [&](int64_t k0) {
    const int64_t row = r0 + ar;
#pragma unroll
    for (int u = 0; u < AE; ++u) {
      const int64_t k = k0 + ak + u;
      ra[u] = (row < Mr && k < K) ? A[row * lda + k] : (T)0;
    }
    const int64_t kb = k0 + bkr;
#pragma unroll
    for (int u = 0; u < BE; ++u) {
      const int64_t c = c0 + bc + u;
      rb[u] = (kb < K && c < N) ? B[kb * ldb + c] : (T)0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < AE; ++u) As[buf][ar * LDA + ak + u] = ra[u];
#pragma unroll
    for (int u = 0; u < BE; ++u) Bs[buf][bkr * LDB + bc + u] = rb[u];
  };
  typename M::Out acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;
  const int64_t np = (K + BK - 1) / BK;
  load(0);
  store(0);
  __syncthreads();
  for (int64_t p = 0; p < np; ++p) {
    const int buf = (int)(p & 1);
    if (p + 1 < np) load((p + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      typename M::Frag fa[4], fb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) fa[i] = As[buf][(wm + 16 * i + li) * LDA + ks * 4 + g];
#pragma unroll
      for (int j = 0; j < 4; ++j) fb[j] = Bs[buf][(ks * 4 + g) * LDB + wn + 16 * j + li];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = M::mma(fa[i], fb[j], acc[i][j]);
    }
    if (p + 1 < np) store(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + wm + 16 * i + M::orow(g, r);
      if (row >= Mr) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t c = c0 + wn + 16 * j + li;
        if (c < N) {
          T *d = out + row * ldc + c;
          const T x = (T)acc[i][j][r];
          *d = accumulate ? *d + x : x;
        }
      }
    }
}

// The same products with BF16 operands on 16x16x32 BF16 MFMA (FP32
// accumulation), for the BF16 sigma.  Both operands are BF16 with k
// contiguous and rows padded with zeros to a multiple of 64 (ld):
// out[r][c] = sum_k A'[r][k] B'[c][k].  Alpha part: A' = H_alpha without
// diagonal, B' = C^T; beta part: A' = C, B' = H_beta without diagonal
// (symmetric, so its rows are its columns).  The padding makes every K
// panel whole and every row 16-byte aligned, so staging is 16-byte vector
// loads with no bounds tests (rows past the end read a clamped valid row
// and are masked at the store).  The epilogue adds the diagonal term in
// FP32 from the FP32 vector: C[r][c] * dd[r] (DSIDE 0) or C[r][c] * dd[c]
// (DSIDE 1).  128 x 256 tiles on 8 waves, K panels of 64.
template <int DSIDE>
__global__ __launch_bounds__(512) void k_gemm_bf16(
    int64_t Mr, int64_t N, int64_t Kp, const __bf16 *__restrict__ Ab, int64_t lda, int64_t sA,
    const __bf16 *__restrict__ Bb, int64_t ldb, int64_t sB, const float *__restrict__ C,
    int64_t sCin, const float *__restrict__ dd, float *__restrict__ out, int64_t ldc, int64_t sC,
    int accumulate, int64_t tiles_n, int64_t per_xcd, int64_t total) {
  constexpr int WM = 2, WN = 4, BM = 64 * WM, BN = 64 * WN, BK = 64, NT = 64 * WM * WN;
  constexpr int LD = BK + 8;  // 144-byte rows: fragments stay 16-byte aligned
  constexpr int AV = BM * BK / NT / 8, BV = BN * BK / NT / 8;  // 16-byte vectors per thread: 2, 4
  __shared__ __align__(16) __bf16 As[2][BM * LD];
  __shared__ __align__(16) __bf16 Bs[2][BN * LD];
  const int64_t b = blockIdx.x;
  const int64_t w = (b & 7) * per_xcd + (b >> 3);
  if (w >= total) return;
  const int64_t tm = w / tiles_n, tn = w - tm * tiles_n;
  const int64_t r0 = tm * BM, c0 = tn * BN;
  const int64_t v = blockIdx.y;
  Ab += v * sA;
  Bb += v * sB;
  C += v * sCin;
  out += v * sC;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int wm = (wave / WN) * 64, wn = (wave % WN) * 64;
  // A' panel: thread -> row ar, 8 AV consecutive k from ak; B' likewise
  const int ar = tid / (BK / (8 * AV)), ak = (tid % (BK / (8 * AV))) * 8 * AV;
  const int br = tid / (BK / (8 * BV)), bk = (tid % (BK / (8 * BV))) * 8 * BV;
  const int64_t arow = r0 + ar < Mr ? r0 + ar : Mr - 1;
  const int64_t brow = c0 + br < N ? c0 + br : N - 1;
  const uint4 *pa = reinterpret_cast<const uint4 *>(Ab + arow * lda + ak);
  const uint4 *pb = reinterpret_cast<const uint4 *>(Bb + brow * ldb + bk);
  uint4 ra[AV], rb[BV];
  auto load = [&](int64_t p) {
#pragma unroll
    for (int u = 0; u < AV; ++u) ra[u] = pa[p * (BK / 8) + u];
#pragma unroll
    for (int u = 0; u < BV; ++u) rb[u] = pb[p * (BK / 8) + u];
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < AV; ++u) *reinterpret_cast<uint4 *>(&As[buf][ar * LD + ak + 8 * u]) = ra[u];
#pragma unroll
    for (int u = 0; u < BV; ++u) *reinterpret_cast<uint4 *>(&Bs[buf][br * LD + bk + 8 * u]) = rb[u];
  };
  f4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.0f;
  const int64_t np = Kp / BK;
  load(0);
  store(0);
  __syncthreads();
  for (int64_t p = 0; p < np; ++p) {
    const int buf = (int)(p & 1);
    if (p + 1 < np) load(p + 1);
#pragma unroll
    for (int ks = 0; ks < BK / 32; ++ks) {
      bf8_t fa[4], fb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        fa[i] = *reinterpret_cast<const bf8_t *>(&As[buf][(wm + 16 * i + li) * LD + ks * 32 + g * 8]);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        fb[j] = *reinterpret_cast<const bf8_t *>(&Bs[buf][(wn + 16 * j + li) * LD + ks * 32 + g * 8]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
    }
    if (p + 1 < np) store(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + wm + 16 * i + 4 * g + r;
      if (row >= Mr) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t c = c0 + wn + 16 * j + li;
        if (c < N) {
          const float x = acc[i][j][r] + C[row * ldc + c] * (DSIDE == 0 ? dd[row] : dd[c]);
          float *d = out + row * ldc + c;
          *d = accumulate ? *d + x : x;
        }
      }
    }
}

// BF16 copies of an [R][C] FP32 matrix (per vector z) with rows padded with
// zeros to ld: transposed (dst[c][r], ld >= R, for the alpha part) or not
// (dst[r][c], ld >= C, for the beta part).
template <bool TRANS>
__global__ void k_to_bf16(const float *__restrict__ src, __bf16 *__restrict__ dst, int64_t R,
                          int64_t C, int64_t ld) {
  __shared__ float tile[TT][TT + 1];
  const int64_t vo = (int64_t)blockIdx.z * R * C;
  const int64_t vd = (int64_t)blockIdx.z * (TRANS ? C : R) * ld;
  const int64_t r0 = (int64_t)blockIdx.y * TT, c0 = (int64_t)blockIdx.x * TT;
  for (int i = threadIdx.y; i < TT; i += blockDim.y) {
    const int64_t r = r0 + i, c = c0 + threadIdx.x;
    tile[i][threadIdx.x] = (r < R && c < C) ? src[vo + r * C + c] : 0.0f;
  }
  __syncthreads();
  for (int i = threadIdx.y; i < TT; i += blockDim.y) {
    if (TRANS) {
      const int64_t c = c0 + i, r = r0 + threadIdx.x;  // dst row c, column r (< ld)
      if (c < C && r < ld) dst[vd + c * ld + r] = (__bf16)tile[threadIdx.x][i];
    } else {
      const int64_t r = r0 + i, c = c0 + threadIdx.x;
      if (r < R && c < ld) dst[vd + r * ld + c] = (__bf16)tile[i][threadIdx.x];
    }
  }
}

// One wave per list row r; each lane owns VC columns c, c + 64, ... so that
// every load instruction of the wave reads 64 consecutive elements.  Work
// items (row group, column tile) are numbered column-tile-major and dealt to
// the 8 XCDs in contiguous ranges (workgroup b runs on XCD b % 8), so each
// XCD streams its own column tiles and its L2 holds one tile's source rows.
template <typename T, typename V, int WAVES, int VC>
__global__ __launch_bounds__(64 * WAVES) void k_same(
    const int32_t *__restrict__ fcol, const V *__restrict__ fval, int nf, int64_t R, int64_t C,
    const T *__restrict__ src, T *__restrict__ dst, int accumulate, int64_t rgroups,
    int64_t per_xcd, int64_t total) {
  const int lane = threadIdx.x & 63;
  const int64_t b = blockIdx.x;
  const int64_t w = (b & 7) * per_xcd + (b >> 3);
  if (w >= total) return;
  const int64_t ct = w / rgroups, rg = w - ct * rgroups;
  const int64_t r = __builtin_amdgcn_readfirstlane((int)(rg * WAVES + (threadIdx.x >> 6)));
  if (r >= R) return;
  const int64_t vo = (int64_t)blockIdx.z * R * C;
  const int64_t c0 = ct * 64 * VC + lane;
  const T *__restrict__ s[VC];
#pragma unroll
  for (int u = 0; u < VC; ++u) {
    int64_t c = c0 + 64 * u;
    s[u] = src + vo + (c < C ? c : C - 1);
  }
  const int32_t *__restrict__ col = fcol + r * nf;
  const V *__restrict__ val = fval + r * nf;
  T acc[VC];
#pragma unroll
  for (int u = 0; u < VC; ++u) acc[u] = 0;
  constexpr int UN = 8;
  int e = 0;
  for (; e + UN <= nf; e += UN) {
    T v[UN][VC];
#pragma unroll
    for (int k = 0; k < UN; ++k) {
      const int64_t off = (int64_t)col[e + k] * C;
#pragma unroll
      for (int u = 0; u < VC; ++u) v[k][u] = s[u][off];
    }
#pragma unroll
    for (int k = 0; k < UN; ++k) {
      const T f = (T)val[e + k];
#pragma unroll
      for (int u = 0; u < VC; ++u) acc[u] += f * v[k][u];
    }
  }
  for (; e < nf; ++e) {
    const int64_t off = (int64_t)col[e] * C;
    const T f = (T)val[e];
#pragma unroll
    for (int u = 0; u < VC; ++u) acc[u] += f * s[u][off];
  }
#pragma unroll
  for (int u = 0; u < VC; ++u) {
    int64_t c = c0 + 64 * u;
    if (c < C) {
      T *d = dst + vo + r * C + c;
      *d = accumulate ? *d + acc[u] : acc[u];
    }
  }
}

// Fixed-point scale of the FP64 opposite-spin scatter for output row ia:
// every partial sum of sigma's row is at most wbound * max_e max |C[J_e][.]|
// (s_beta contributions per element, each at most max_kl sum |W[kl][.]| times
// the largest C entry the row gathers); the power-of-two scale puts that
// bound below 2^62.  bad: a non-finite C row (the result becomes NaN).
// Called by every thread of the workgroup (it holds a barrier).
template <int NW>
__device__ inline void fix_scale(const double *__restrict__ rowmax, const Ent *__restrict__ taba,
                                 int64_t ia, int s, int64_t nsa, double wbound, double *wmax,
                                 double &scale, double &inv, bool &bad) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double m = 0.0;
  for (int e = tid; e < s; e += 64 * NW) {
    const double r = rowmax[(int64_t)blockIdx.y * nsa + taba[ia * s + e].J];
    m = (r > m || r != r) ? r : m;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double r = __shfl_xor(m, o);
    m = (r > m || r != r) ? r : m;
  }
  if (lane == 0) wmax[wave] = m;
  __syncthreads();
  m = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) m = (wmax[w] > m || wmax[w] != wmax[w]) ? wmax[w] : m;
  fix_scale_from_bound(wbound * m, scale, inv, bad);
}

// Dynamic LDS of the opposite-spin kernels: 160 KB less the static
// per-wave scale slots of the FP64 fixed-point scatter (NW doubles).
constexpr size_t kOppLdsCap = 160 * 1024 - 256;

constexpr int32_t kPadEntry = -1;  // K padding: zero column of A

// Opposite-spin contraction, one output row Ia (of one vector) per
// workgroup of NW waves.
//   M[kl][J] = sum_e sign_e (kl|kl_e) C[J_e][J]     e over the alpha
//              single excitations (p_e, q_e, J_e, sign_e) of Ia (incl. diagonal)
//   sigma[Ia][I'] += sign' M[kl][J]                 for E_kl or E_lk |J> = sign' |I'>
// LDS (dynamic): acc[nsb + 64] | Ws[ngroups*MG*16][KW + PAD] | eoff[nkc*KW] | eW[nkc*KW]
//   acc  sigma's row Ia; the 64 extra slots absorb the lanes whose pair
//        code is invalid, so the scatter needs no branch
//   Ws   A tile of one K chunk: sign_e (kl|kl_e), zero for padded rows / K
//   eoff row offset J_e * nsb of the C row feeding K element e; padded K
//        elements point at row Ia itself (in its own list as the diagonal
//        excitation, so a non-finite value there makes the row NaN anyway)
// Each wave owns 16-column tiles J0 = 16 (wave + NW i).  It gathers the B
// fragment C[J_e][J0 + li] straight from global memory into registers (the
// next tile's fragment is fetched before the current tile's MFMAs), runs all
// M tiles of its group, and scatters through the packed pair codes.  K and M
// are padded to compile-time tile counts, so the inner loops carry no bound
// checks; no workgroup barrier sits inside the column loop.  c (type TC,
// row stride ldc) is the vector itself, or for the BF16 flavour its BF16
// copy, which halves the bytes of the gathers.
template <typename M, typename T, typename TC, int MG, int KS, bool AREG, int NW, bool FIXT>
__global__ __launch_bounds__(64 * NW) void k_opp(
    int64_t nsa, int64_t nsb, int64_t nsb_pad, int s, int npair, int ngroups, int nkc,
    const float *__restrict__ Wf, const double *__restrict__ Wd, const Ent *__restrict__ taba,
    const uint4 *__restrict__ quads, const TC *__restrict__ c, int64_t ldc,
    T *__restrict__ sigma, int64_t per_xcd, const double *__restrict__ rowmax, double wbound) {
  using A = typename M::A;
  using Acc = typename M::Acc;
  using Frag = typename M::Frag;
  constexpr int KW = KS * M::KSTEP;
  constexpr int LDW = KW + M::PAD;
  constexpr int GROWS = MG * 16;
  // FIXT (FP64, the default): sigma's row accumulates in 64-bit fixed point
  // (integer LDS atomics, exact and order-independent), so the result does
  // not depend on the order in which waves scatter
  constexpr bool FIX = FIXT && std::is_same<M, MF64>::value;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double wmax[NW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // rows are dealt to the 8 XCDs in contiguous ranges (workgroup b runs on
  // XCD b % 8): neighbouring alpha strings share most of their excited
  // strings J_e, so the workgroups of one XCD find the same C rows in its L2
  const int64_t ia = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (ia >= nsa) return;
  const int64_t vo = (int64_t)blockIdx.y * nsa * nsb;
  const int MROWS = ngroups * GROWS;
  const int ktot = nkc * KW;
  Acc *acc = reinterpret_cast<Acc *>(smem);
  size_t off = ((size_t)(nsb + 64) * sizeof(Acc) + 15) & ~(size_t)15;
  A *Ws = reinterpret_cast<A *>(smem + off);
  off += (((size_t)MROWS * LDW * sizeof(A)) + 15) & ~(size_t)15;
  uint32_t *eoff = reinterpret_cast<uint32_t *>(smem + off);
  off += (size_t)ktot * sizeof(uint32_t);
  int32_t *eW = reinterpret_cast<int32_t *>(smem + off);

  for (int e = tid; e < ktot; e += 64 * NW) {
    if (e < s) {
      Ent t = taba[ia * s + e];
      eoff[e] = (uint32_t)t.J * (uint32_t)ldc;
      int kl = pair_index(t.p, t.q);
      eW[e] = t.sign < 0 ? (kl | (int32_t)0x80000000) : kl;
    } else {
      eoff[e] = (uint32_t)ia * (uint32_t)ldc;  // any valid row: its A column is zero
      eW[e] = kPadEntry;
    }
  }
  for (int64_t j = tid; j < nsb + 64; j += 64 * NW) acc[j] = (Acc)0;
  double fscale = 1.0, finv = 1.0;
  bool fbad = false;
  if constexpr (FIX) fix_scale<NW>(rowmax, taba, ia, s, nsa, wbound, wmax, fscale, finv, fbad);

  const TC *__restrict__ cv = c + (int64_t)blockIdx.y * nsa * ldc;
  const uint32_t nsb32 = (uint32_t)nsb;
  const uint32_t pstride = (uint32_t)nsb_pad;
  const int njt = (int)((nsb + 15) / 16);
  const int g = lane >> 4;
  const int li = lane & 15;

  for (int kc = 0; kc < nkc; ++kc) {
    __syncthreads();  // entries ready; the previous chunk's Ws is no longer read
    for (int idx = tid; idx < MROWS * KW; idx += 64 * NW) {
      const int row = idx / KW, k = idx - row * KW;
      const int w = eW[kc * KW + k];
      A v = M::cvt(0.0f);
      if (w != kPadEntry && row < npair) {
        const int kl = w & 0x7fffffff;
        double x = Wd ? Wd[(int64_t)row * npair + kl] : (double)Wf[(int64_t)row * npair + kl];
        if constexpr (FIX) x *= fscale;  // a power of two: exact; M comes out in fixed-point units
        v = M::cvt(w < 0 ? -x : x);
      }
      Ws[row * LDW + k] = v;
    }
    __syncthreads();
    uint32_t boff[KS][M::KPL];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int t = 0; t < M::KPL; ++t) boff[ks][t] = eoff[kc * KW + ks * M::KSTEP + g * M::KPL + t];
    Frag areg[AREG ? MG : 1][AREG ? KS : 1];
    if constexpr (AREG) {
#pragma unroll
      for (int u = 0; u < MG; ++u)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
          areg[u][ks] = M::load_a(&Ws[(u * 16 + li) * LDW + ks * M::KSTEP + g * M::KPL]);
    }
    // Per column tile: load this tile's pair codes, then prefetch the next
    // tile's B fragments (unconditionally: past the last tile a clamped,
    // valid column is fetched and never used), then multiply and scatter.
    // Loads complete in issue order, so the scatter's wait for the codes
    // leaves the prefetch in flight and the codes' latency hides behind the
    // MFMAs.  Pair-table rows are padded to whole 16-column tiles with
    // invalid codes, and out-of-range B columns are clamped, so no lane
    // needs a column test.
    int jt = wave;
    Frag bn[KS];
    {
      const uint32_t J = (uint32_t)(jt * 16 + li);
      const uint32_t jl = J < nsb32 ? J : nsb32 - 1;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) bn[ks] = M::load_b(cv, boff[ks], jl);
    }
    for (; jt < njt; jt += NW) {
      const uint32_t J = (uint32_t)(jt * 16 + li);
      Frag b[KS];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) b[ks] = bn[ks];
      for (int grp = 0; grp < ngroups; ++grp) {
        uint4 code[MG];
#pragma unroll
        for (int u = 0; u < MG; ++u)
          code[u] = quads[((uint32_t)(grp * MG + u) * 4u + (uint32_t)g) * pstride + J];
        if (grp == 0) {
          const uint32_t Jn = (uint32_t)((jt + NW) * 16 + li);
          const uint32_t jn = Jn < nsb32 ? Jn : nsb32 - 1;
#pragma unroll
          for (int ks = 0; ks < KS; ++ks) bn[ks] = M::load_b(cv, boff[ks], jn);
        }
        // keep the loads above ahead of the MFMAs below (issue order matters)
        __builtin_amdgcn_sched_barrier(0);
        typename M::Out out[MG];
#pragma unroll
        for (int u = 0; u < MG; ++u)
#pragma unroll
          for (int r = 0; r < 4; ++r) out[u][r] = 0;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
          for (int u = 0; u < MG; ++u) {
            Frag a;
            if constexpr (AREG)
              a = areg[u][ks];
            else
              a = M::load_a(&Ws[(grp * GROWS + u * 16 + li) * LDW + ks * M::KSTEP + g * M::KPL]);
            out[u] = M::mma(a, b[ks], out[u]);
          }
        // only lanes with a valid code scatter (the others are masked off
        // and cost no LDS bandwidth)
#pragma unroll
        for (int u = 0; u < MG; ++u) {
          const uint32_t cds[4] = {code[u].x, code[u].y, code[u].z, code[u].w};
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const uint32_t cd = cds[r];
            if (cd != kInvalid) {
              Acc v = (Acc)out[u][r];
              if (cd & 1u) v = -v;
              scatter_add<FIX>(&acc[cd >> 1], v);
            }
          }
        }
      }
    }
  }
  __syncthreads();
  T *__restrict__ sv = sigma + vo + ia * nsb;
  for (int64_t j = tid; j < nsb; j += 64 * NW) sv[j] += row_value<FIX, T>(acc, j, finv, fbad);
}

// max |C[J][.]| of every alpha row J (and vector): the fixed-point scale of
// the FP64 opposite-spin scatter; NaN if the row holds a NaN
__global__ __launch_bounds__(256) void k_rowmax(const double *__restrict__ c, int64_t nsa,
                                                int64_t nsb, double *__restrict__ out) {
  __shared__ double red[4];
  const int64_t J = blockIdx.x;
  const double *row = c + ((int64_t)blockIdx.y * nsa + J) * nsb;
  double m = 0.0;
  for (int64_t j = threadIdx.x; j < nsb; j += 256) {
    const double a = fabs(row[j]);
    m = (a > m || a != a) ? a : m;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double r = __shfl_xor(m, o);
    m = (r > m || r != r) ? r : m;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int w = 1; w < 4; ++w) r = (red[w] > r || red[w] != red[w]) ? red[w] : r;
    out[(int64_t)blockIdx.y * nsa + J] = r;
  }
}

struct OppPlan {
  int MG, KS, ngroups, nkc;
  size_t lds;
};

template <typename M>
size_t opp_lds(int64_t nsb, int MG, int KS, int ngroups, int nkc) {
  const int KW = KS * M::KSTEP, LDW = KW + M::PAD;
  size_t b = ((size_t)(nsb + 64) * sizeof(typename M::Acc) + 15) & ~(size_t)15;
  b += (((size_t)ngroups * MG * 16 * LDW * sizeof(typename M::A)) + 15) & ~(size_t)15;
  b += (size_t)nkc * KW * 8;
  return b;
}

template <typename M>
int plan_opp(sbci_ctx *ctx, const int *mg_options, int nmg, const int *ks_options, int nks,
             OppPlan &p) {
  const SpinTables &A = ctx->A, &B = ctx->B;
  const int Mt = (ctx->npair + 15) / 16;
  const int kst = (A.s + M::KSTEP - 1) / M::KSTEP;
  const size_t cap = kOppLdsCap;
  // (M tiles per group, k-steps per chunk) with the least padded MFMA work
  // per column tile, ngroups * MG * nkc * KS, among those that fit in LDS;
  // ties: fewer K chunks (fewer barriers), then fewer groups
  p.MG = p.KS = 0;
  int64_t best = -1;
  for (int i = 0; i < nmg; ++i) {
    const int mg = mg_options[i], ng = (Mt + mg - 1) / mg;
    if (ng * mg * 16 > ctx->npair_pad) continue;
    for (int j = 0; j < nks; ++j) {
      const int ks = ks_options[j], nkc = (kst + ks - 1) / ks;
      if (opp_lds<M>(B.ns, mg, ks, ng, nkc) > cap) continue;
      // the FP64 tile of 9 x 14 needs more than 256 VGPRs (spills)
      if (std::is_same<typename M::A, double>::value && mg * ks > 100) continue;
      const int64_t work = (int64_t)ng * mg * nkc * ks;
      if (best < 0 || work < best || (work == best && nkc < p.nkc) ||
          (work == best && nkc == p.nkc && ng < p.ngroups)) {
        best = work;
        p.MG = mg;
        p.KS = ks;
        p.nkc = nkc;
        p.ngroups = ng;
      }
    }
  }
  if (p.KS == 0)
    return set_error(SBCI_EINVAL, "opposite-spin sigma: beta string count too large for LDS");
  p.lds = opp_lds<M>(B.ns, p.MG, p.KS, p.ngroups, p.nkc);
  return SBCI_OK;
}

template <typename M, typename T, int MG, int KS, bool AREG, typename TC>
void launch_opp_k(sbci_ctx *ctx, const OppPlan &p, dim3 grid, const float *Wf, const double *Wd,
                  const TC *c, int64_t ldc, T *out, const double *rowmax) {
  const SpinTables &A = ctx->A, &B = ctx->B;
  constexpr int NW = 8;
  auto launch = [&](auto kern) {
    static bool attr = false;
    if (!attr) {
      hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)kOppLdsCap);
      attr = true;
    }
    kern<<<grid, 64 * NW, p.lds, ctx->stream>>>(
        A.ns, B.ns, B.ns_pad, A.s, ctx->npair, p.ngroups, p.nkc, Wf, Wd, A.tab,
        std::is_same<typename M::A, double>::value ? B.quad_s : B.quad_r, c, ldc, out,
        (int64_t)(grid.x / 8), rowmax, ctx->opp_wbound);
  };
  if (std::is_same<M, MF64>::value && ctx->deterministic)
    launch(k_opp<M, T, TC, MG, KS, AREG, NW, std::is_same<M, MF64>::value>);
  else
    launch(k_opp<M, T, TC, MG, KS, AREG, NW, false>);
}

template <typename M, typename T, int MG, typename TC>
void dispatch_ks(sbci_ctx *ctx, const OppPlan &p, dim3 grid, const float *Wf, const double *Wd,
                 const TC *c, int64_t ldc, T *out, const double *rowmax) {
  if constexpr (M::KPL == 8) {
    // A fragments in registers when they are few enough (MG * KS <= 18)
    const bool areg = p.ngroups == 1 && MG * p.KS <= 18;
    if (p.KS == 1) {
      if (areg) launch_opp_k<M, T, MG, 1, true, TC>(ctx, p, grid, Wf, Wd, c, ldc, out, rowmax);
      else launch_opp_k<M, T, MG, 1, false, TC>(ctx, p, grid, Wf, Wd, c, ldc, out, rowmax);
    } else if (p.KS == 2) {
      if (areg) launch_opp_k<M, T, MG, 2, true, TC>(ctx, p, grid, Wf, Wd, c, ldc, out, rowmax);
      else launch_opp_k<M, T, MG, 2, false, TC>(ctx, p, grid, Wf, Wd, c, ldc, out, rowmax);
    } else {
      if (areg) launch_opp_k<M, T, MG, 3, true, TC>(ctx, p, grid, Wf, Wd, c, ldc, out, rowmax);
      else launch_opp_k<M, T, MG, 3, false, TC>(ctx, p, grid, Wf, Wd, c, ldc, out, rowmax);
    }
  } else {
    if constexpr (std::is_same<typename M::A, double>::value) {
      if (p.KS == 4) launch_opp_k<M, T, MG, 4, false, TC>(ctx, p, grid, Wf, Wd, c, ldc, out, rowmax);
      else if (p.KS == 6) launch_opp_k<M, T, MG, 6, false, TC>(ctx, p, grid, Wf, Wd, c, ldc, out, rowmax);
      else if (p.KS == 7) launch_opp_k<M, T, MG, 7, false, TC>(ctx, p, grid, Wf, Wd, c, ldc, out, rowmax);
      else if (p.KS == 9) launch_opp_k<M, T, MG, 9, false, TC>(ctx, p, grid, Wf, Wd, c, ldc, out, rowmax);
      else launch_opp_k<M, T, MG, 14, false, TC>(ctx, p, grid, Wf, Wd, c, ldc, out, rowmax);
    } else {
      if (p.KS == 8) launch_opp_k<M, T, MG, 8, false, TC>(ctx, p, grid, Wf, Wd, c, ldc, out, rowmax);
      else if (p.KS == 9) launch_opp_k<M, T, MG, 9, false, TC>(ctx, p, grid, Wf, Wd, c, ldc, out, rowmax);
      else launch_opp_k<M, T, MG, 14, false, TC>(ctx, p, grid, Wf, Wd, c, ldc, out, rowmax);
    }
  }
}

template <typename M, typename T, typename TC>
int launch_opp_pair(sbci_ctx *ctx, const OppPlan &p, const TC *c, int64_t ldc, T *out, int nvec,
                    double *rmax) {
  const SpinTables &A = ctx->A;
  const float *Wf = nullptr;
  const double *Wd = nullptr;
  if constexpr (std::is_same<typename M::A, double>::value) Wd = ctx->W64; else Wf = ctx->W32;
  const int64_t per_xcd = (A.ns + 7) / 8;
  dim3 grid((unsigned)(per_xcd * 8), (unsigned)nvec);
  if constexpr (std::is_same<M, MF64>::value) {
    if (ctx->deterministic) {
      k_rowmax<<<dim3((unsigned)A.ns, (unsigned)nvec), 256, 0, ctx->stream>>>(
          reinterpret_cast<const double *>(c), A.ns, ldc, rmax);
      SBCI_CHECK_LAUNCH();
    }
  }
  if constexpr (std::is_same<typename M::A, double>::value) {
    if (p.MG == 4) dispatch_ks<M, T, 4, TC>(ctx, p, grid, Wf, Wd, c, ldc, out, rmax);
    else if (p.MG == 5) dispatch_ks<M, T, 5, TC>(ctx, p, grid, Wf, Wd, c, ldc, out, rmax);
    else if (p.MG == 7) dispatch_ks<M, T, 7, TC>(ctx, p, grid, Wf, Wd, c, ldc, out, rmax);
    else dispatch_ks<M, T, 9, TC>(ctx, p, grid, Wf, Wd, c, ldc, out, rmax);
  } else {
    if (p.MG == 4) dispatch_ks<M, T, 4, TC>(ctx, p, grid, Wf, Wd, c, ldc, out, rmax);
    else if (p.MG == 7) dispatch_ks<M, T, 7, TC>(ctx, p, grid, Wf, Wd, c, ldc, out, rmax);
    else dispatch_ks<M, T, 9, TC>(ctx, p, grid, Wf, Wd, c, ldc, out, rmax);
  }
  SBCI_CHECK_LAUNCH();
  return SBCI_OK;
}

// Orbital-grouped opposite-spin contraction, the form for dilute spaces
// (few electrons in many orbitals), where most orbital pairs {k, l} connect
// a string to nothing and k_opp's M[kl][J] is mostly discarded.  E_pq acts
// on a beta string only if it holds q, and then yields a string for every p
// that is q or empty.  For output row Ia and beta orbital q:
//   M_q[p][j] = sum_e sign_e (pq|kl_e) Cq[q][J_e][j]      p = 0..N-1
//   sigma[Ia][I'] += sign' M_q[p][j]   for E_pq colq[q][j] = sign' |I'>
// Cq[q][Ia][j] = C[Ia][colq[q][j]] is gathered once per sigma (k_gather_q),
// so B fragments are contiguous row segments as in k_opp.  Per determinant
// this issues 2 N m_beta s flops (k_opp: 2 npair s; minimum 2 s^2).  Rows
// are dealt to the 8 XCDs in contiguous ranges: neighbouring rows differ in
// one orbital and share many excited strings J_e, so the workgroups of one
// XCD, which sweep q together, find the same Cq rows in its L2.  When
// sigma's row does not fit in LDS, blockIdx.z selects a window of win
// target strings: the workgroup computes every M_q but scatters only the
// targets in its window (nwin windows cost nwin times the MFMA work).
// LDS (dynamic): acc[win + 64] | Ws[MT*16][KW + PAD] | eoff[nkc*KW] | eW[nkc*KW]
template <typename M, typename T, int MT, int KS, int NW, bool FIXT>
__global__ __launch_bounds__(64 * NW) void k_opp_q(
    int64_t nsa, int64_t nsb, int norb, int64_t nq, int64_t nq_pad, int s, int npair, int nkc,
    int64_t per_xcd, int64_t win, const float *__restrict__ Wf, const double *__restrict__ Wd,
    const Ent *__restrict__ taba, const uint4 *__restrict__ quads, const T *__restrict__ cq,
    T *__restrict__ sigma, const double *__restrict__ rowmax, double wbound) {
  using A = typename M::A;
  using Acc = typename M::Acc;
  using Frag = typename M::Frag;
  constexpr int KW = KS * M::KSTEP;
  constexpr int LDW = KW + M::PAD;
  constexpr int ROWS = MT * 16;
  constexpr bool FIX = FIXT && std::is_same<M, MF64>::value;  // fixed-point FP64 scatter (see k_opp)
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double wmax[NW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t ia = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (ia >= nsa) return;  // uniform over the workgroup
  const int64_t vo = (int64_t)blockIdx.y * nsa * nsb;
  const int64_t t0 = (int64_t)blockIdx.z * win;
  const int64_t tlen = t0 >= nsb ? 0 : (nsb - t0 < win ? nsb - t0 : win);
  const uint32_t t032 = (uint32_t)t0, tlen32 = (uint32_t)tlen;
  const int ktot = nkc * KW;
  Acc *acc = reinterpret_cast<Acc *>(smem);
  size_t off = ((size_t)(win + 64) * sizeof(Acc) + 15) & ~(size_t)15;
  A *Ws = reinterpret_cast<A *>(smem + off);
  off += (((size_t)ROWS * LDW * sizeof(A)) + 15) & ~(size_t)15;
  uint32_t *eoff = reinterpret_cast<uint32_t *>(smem + off);
  off += (size_t)ktot * sizeof(uint32_t);
  int32_t *eW = reinterpret_cast<int32_t *>(smem + off);

  const uint32_t nq32 = (uint32_t)nq;
  for (int e = tid; e < ktot; e += 64 * NW) {
    if (e < s) {
      Ent t = taba[ia * s + e];
      eoff[e] = (uint32_t)t.J * nq32;
      int kl = pair_index(t.p, t.q);
      eW[e] = t.sign < 0 ? (kl | (int32_t)0x80000000) : kl;
    } else {
      // the row of the first entry of this K chunk (a row this row gathers,
      // in the same loads: a non-finite value there already makes the row
      // NaN); its A column is zero.  A row outside the list could carry a
      // NaN or Inf into M through 0 * NaN.  Every chunk starts with a real
      // entry, since the chunks cover s entries with less than one chunk of
      // padding.
      eoff[e] = (uint32_t)taba[ia * s + (e / KW) * KW].J * nq32;
      eW[e] = kPadEntry;
    }
  }
  for (int64_t j = tid; j < win + 64; j += 64 * NW) acc[j] = (Acc)0;
  double fscale = 1.0, finv = 1.0;
  bool fbad = false;
  if constexpr (FIX) fix_scale<NW>(rowmax, taba, ia, s, nsa, wbound, wmax, fscale, finv, fbad);

  const int njt = (int)(nq_pad / 16);
  const int g = lane >> 4;
  const int li = lane & 15;
  const uint32_t pstride = (uint32_t)nq_pad;
  // The A tile of chunk (q, kc) is fetched into registers while the previous
  // chunk's MFMAs run, and stored to LDS between two barriers.
  constexpr int NA = (ROWS * KW + 64 * NW - 1) / (64 * NW);
  A va[NA];
  auto fetch_a = [&](int q, int kc) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int idx = tid + i * 64 * NW;
      A v = M::cvt(0.0f);
      if (idx < ROWS * KW) {
        const int p = idx / KW, k = idx - p * KW;
        const int w = eW[kc * KW + k];
        if (w != kPadEntry && p < norb) {
          const int kl = w & 0x7fffffff;
          const int64_t pq = pair_index(p, q);
          double x = Wd ? Wd[pq * npair + kl] : (double)Wf[pq * npair + kl];
          if constexpr (FIX) x *= fscale;  // exact: M in fixed-point units
          v = M::cvt(w < 0 ? -x : x);
        }
      }
      va[i] = v;
    }
  };
  __syncthreads();  // entries ready
  fetch_a(0, 0);
  for (int q = 0; q < norb; ++q) {
    const T *__restrict__ cv = cq + ((int64_t)blockIdx.y * norb + q) * nsa * nq;
    const uint4 *__restrict__ qq = quads + (int64_t)q * MT * 4 * nq_pad;
    for (int kc = 0; kc < nkc; ++kc) {
      __syncthreads();  // the previous A tile is no longer read
#pragma unroll
      for (int i = 0; i < NA; ++i) {
        const int idx = tid + i * 64 * NW;
        if (idx < ROWS * KW) {
          const int p = idx / KW, k = idx - p * KW;
          Ws[p * LDW + k] = va[i];
        }
      }
      __syncthreads();
      {
        const int kn = kc + 1 < nkc ? kc + 1 : 0;
        const int qn = kc + 1 < nkc ? q : q + 1;
        if (qn < norb) fetch_a(qn, kn);
      }
      uint32_t boff[KS][M::KPL];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int t = 0; t < M::KPL; ++t) boff[ks][t] = eoff[kc * KW + ks * M::KSTEP + g * M::KPL + t];
      // As in k_opp: codes of this tile, then the next tile's B fragments
      // (clamped to a valid column past the end), then MFMAs and the
      // scatter.  Columns past nq carry invalid codes.
      int jt = wave;
      Frag bn[KS];
      {
        const uint32_t J = (uint32_t)(jt * 16 + li);
        const uint32_t jl = J < nq32 ? J : nq32 - 1;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) bn[ks] = M::load_b(cv, boff[ks], jl);
      }
      for (; jt < njt; jt += NW) {
        const uint32_t J = (uint32_t)(jt * 16 + li);
        Frag b[KS];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) b[ks] = bn[ks];
        uint4 code[MT];
#pragma unroll
        for (int u = 0; u < MT; ++u) code[u] = qq[((uint32_t)u * 4u + (uint32_t)g) * pstride + J];
        {
          const uint32_t Jn = (uint32_t)((jt + NW) * 16 + li);
          const uint32_t jn = Jn < nq32 ? Jn : nq32 - 1;
#pragma unroll
          for (int ks = 0; ks < KS; ++ks) bn[ks] = M::load_b(cv, boff[ks], jn);
        }
        __builtin_amdgcn_sched_barrier(0);
        typename M::Out out[MT];
#pragma unroll
        for (int u = 0; u < MT; ++u)
#pragma unroll
          for (int r = 0; r < 4; ++r) out[u][r] = 0;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
          for (int u = 0; u < MT; ++u) {
            const Frag a = M::load_a(&Ws[(u * 16 + li) * LDW + ks * M::KSTEP + g * M::KPL]);
            out[u] = M::mma(a, b[ks], out[u]);
          }
#pragma unroll
        for (int u = 0; u < MT; ++u) {
          const uint32_t cds[4] = {code[u].x, code[u].y, code[u].z, code[u].w};
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const uint32_t cd = cds[r];
            const uint32_t tw = (cd >> 1) - t032;  // wraps above tlen if below t0
            if (cd != kInvalid && tw < tlen32) {
              Acc v = (Acc)out[u][r];
              if (cd & 1u) v = -v;
              scatter_add<FIX>(&acc[tw], v);
            }
          }
        }
      }
    }
  }
  __syncthreads();
  T *__restrict__ sv = sigma + vo + ia * nsb + t0;
  for (int64_t j = tid; j < tlen; j += 64 * NW) sv[j] += row_value<FIX, T>(acc, j, finv, fbad);
}

// cq[v][q][Ia][j] = c[v][Ia][colq[q][j]]; blocks of one row Ia are adjacent
// in launch order, so the row is read from HBM about once.
template <typename T>
__global__ void k_gather_q(const T *__restrict__ c, T *__restrict__ cq,
                           const int32_t *__restrict__ colq, int64_t nsa, int64_t nsb, int norb,
                           int64_t nq, int64_t jblocks) {
  const int64_t b = blockIdx.x;
  const int64_t ia = b / (norb * jblocks);
  const int64_t r = b - ia * norb * jblocks;
  const int q = (int)(r / jblocks);
  const int64_t j = (r - (int64_t)q * jblocks) * blockDim.x + threadIdx.x;
  if (j >= nq) return;
  const int64_t v = blockIdx.y;
  cq[((v * norb + q) * nsa + ia) * nq + j] = c[v * nsa * nsb + ia * nsb + colq[(int64_t)q * nq + j]];
}

struct OppQPlan {
  int KS = 0, nkc = 0;
  int64_t win = 0, nwin = 0;  // target window of sigma's row and window count
  size_t lds = 0;
};

template <typename M>
size_t oppq_lds(int64_t win, int MT, int KS, int nkc) {
  const int KW = KS * M::KSTEP, LDW = KW + M::PAD;
  size_t b = ((size_t)(win + 64) * sizeof(typename M::Acc) + 15) & ~(size_t)15;
  b += (((size_t)MT * 16 * LDW * sizeof(typename M::A)) + 15) & ~(size_t)15;
  b += (size_t)nkc * KW * 8;
  return b;
}

// K tile (k-steps per chunk) and target windows: the fewest windows that
// fit in LDS (at least min_win), then the least K padding (ties: fewer
// chunks); false if nothing fits.
template <typename M>
bool plan_opp_q(const sbci_ctx *ctx, OppQPlan &p, int64_t min_win) {
  const SpinTables &A = ctx->A, &B = ctx->B;
  if (B.nq == 0 || B.mt < 1 || B.mt > 4) return false;
  static const int ks_w[3] = {9, 12, 17};
  static const int ks_b[3] = {1, 3, 5};
  const int *opts = M::KPL == 8 ? ks_b : ks_w;
  const int kst = (A.s + M::KSTEP - 1) / M::KSTEP;
  const size_t cap = kOppLdsCap;
  p = OppQPlan();
  int64_t best = -1;
  for (int i = 0; i < 3; ++i) {
    const int ks = opts[i], nkc = (kst + ks - 1) / ks;
    const size_t fixed = oppq_lds<M>(0, B.mt, ks, nkc) + 16;
    if (fixed + 128 * sizeof(typename M::Acc) > cap) continue;
    const int64_t wmax = (int64_t)((cap - fixed) / sizeof(typename M::Acc)) - 64;
    int64_t nwin = (B.ns + wmax - 1) / wmax;
    if (nwin < min_win) nwin = min_win;
    if (nwin > B.ns) nwin = B.ns;
    const int64_t cost = nwin * 4096 + (int64_t)nkc * ks;  // windows first, then K padding
    if (best < 0 || cost < best || (cost == best && nkc < p.nkc)) {
      best = cost;
      p.KS = ks;
      p.nkc = nkc;
      p.win = (B.ns + nwin - 1) / nwin;
      p.nwin = (B.ns + p.win - 1) / p.win;  // every window non-empty
    }
  }
  if (p.KS == 0 || p.nwin > 65535) return false;
  p.lds = oppq_lds<M>(p.win, B.mt, p.KS, p.nkc);
  return p.lds <= cap;
}

template <typename M, typename T, int MT, int KS>
int launch_opp_q_k(sbci_ctx *ctx, const OppQPlan &p, const float *Wf, const double *Wd,
                   const T *cq, T *out, int nvec, const double *rmax) {
  const SpinTables &A = ctx->A, &B = ctx->B;
  constexpr int NW = 8;
  const uint4 *quads = std::is_same<typename M::A, double>::value ? B.qquad_s : B.qquad_r;
  const int64_t per_xcd = (A.ns + 7) / 8;
  auto launch = [&](auto kern) -> int {
    static bool attr = false;
    if (!attr) {
      SBCI_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)kOppLdsCap));
      attr = true;
    }
    kern<<<dim3((unsigned)(per_xcd * 8), (unsigned)nvec, (unsigned)p.nwin), 64 * NW, p.lds,
           ctx->stream>>>(A.ns, B.ns, ctx->norb, B.nq, B.nq_pad, A.s, ctx->npair, p.nkc, per_xcd,
                          p.win, Wf, Wd, A.tab, quads, cq, out, rmax, ctx->opp_wbound);
    return SBCI_OK;
  };
  if (std::is_same<M, MF64>::value && ctx->deterministic)
    SBCI_TRY(launch(k_opp_q<M, T, MT, KS, NW, std::is_same<M, MF64>::value>));
  else
    SBCI_TRY(launch(k_opp_q<M, T, MT, KS, NW, false>));
  SBCI_CHECK_LAUNCH();
  return SBCI_OK;
}

template <typename M, typename T, int MT>
int dispatch_q_ks(sbci_ctx *ctx, const OppQPlan &p, const float *Wf, const double *Wd, const T *cq,
                  T *out, int nvec, const double *rmax) {
  if constexpr (M::KPL == 8) {
    if (p.KS == 1) return launch_opp_q_k<M, T, MT, 1>(ctx, p, Wf, Wd, cq, out, nvec, rmax);
    if (p.KS == 3) return launch_opp_q_k<M, T, MT, 3>(ctx, p, Wf, Wd, cq, out, nvec, rmax);
    return launch_opp_q_k<M, T, MT, 5>(ctx, p, Wf, Wd, cq, out, nvec, rmax);
  } else {
    if (p.KS == 9) return launch_opp_q_k<M, T, MT, 9>(ctx, p, Wf, Wd, cq, out, nvec, rmax);
    if (p.KS == 12) return launch_opp_q_k<M, T, MT, 12>(ctx, p, Wf, Wd, cq, out, nvec, rmax);
    return launch_opp_q_k<M, T, MT, 17>(ctx, p, Wf, Wd, cq, out, nvec, rmax);
  }
}

template <typename M, typename T>
int launch_opp_q(sbci_ctx *ctx, const OppQPlan &p, const T *c, T *out, int nvec, double *rmax) {
  const SpinTables &A = ctx->A, &B = ctx->B;
  const int n = ctx->norb;
  const size_t bytes = sizeof(T) * (size_t)nvec * n * A.ns * B.nq;
  SBCI_TRY(ensure(ctx->ws_q, bytes));
  T *cq = static_cast<T *>(ctx->ws_q.ptr);
  const int64_t jblocks = (B.nq + 255) / 256;
  const int64_t nblk = A.ns * n * jblocks;
  if (nblk >= ((int64_t)1 << 31)) return set_error(SBCI_EINVAL, "opposite-spin sigma: grid too large");
  k_gather_q<T><<<dim3((unsigned)nblk, (unsigned)nvec), 256, 0, ctx->stream>>>(c, cq, B.colq, A.ns,
                                                                             B.ns, n, B.nq, jblocks);
  SBCI_CHECK_LAUNCH();
  const float *Wf = nullptr;
  const double *Wd = nullptr;
  if constexpr (std::is_same<typename M::A, double>::value) Wd = ctx->W64; else Wf = ctx->W32;
  if constexpr (std::is_same<M, MF64>::value) {
    if (ctx->deterministic) {
      k_rowmax<<<dim3((unsigned)A.ns, (unsigned)nvec), 256, 0, ctx->stream>>>(
          reinterpret_cast<const double *>(c), A.ns, B.ns, rmax);
      SBCI_CHECK_LAUNCH();
    }
  }
  switch (B.mt) {
    case 1: return dispatch_q_ks<M, T, 1>(ctx, p, Wf, Wd, cq, out, nvec, rmax);
    case 2: return dispatch_q_ks<M, T, 2>(ctx, p, Wf, Wd, cq, out, nvec, rmax);
    case 3: return dispatch_q_ks<M, T, 3>(ctx, p, Wf, Wd, cq, out, nvec, rmax);
    default: return dispatch_q_ks<M, T, 4>(ctx, p, Wf, Wd, cq, out, nvec, rmax);
  }
}

// Opposite-spin form for this context and flavour: the pair form (k_opp) or
// the orbital-grouped form (k_opp_q).  Automatic choice: the orbital form
// when the pair form does not fit in LDS, or when it issues at most 2/3 of
// the pair form's MFMA tiles (its B operand is read m_beta times per row).
template <typename M>
int choose_opp(sbci_ctx *ctx, int &form, OppPlan &pp, OppQPlan &pq) {
  const SpinTables &A = ctx->A, &B = ctx->B;
  const int64_t min_win = ctx->opp_form == SBCI_OPP_ORBITAL_WINDOWED ? 2 : 1;
  const bool qok = plan_opp_q<M>(ctx, pq, min_win) && (uint64_t)A.ns * (uint64_t)B.nq < (1ull << 32);
  bool pok = false;
  {
    // K tiles (k-steps per chunk) offered to the pair planner; the register
    // budget of two waves per SIMD bounds them (B fragments double-buffered)
    static const int ks_d[5] = {4, 6, 7, 9, 14};
    static const int ks_f[3] = {8, 9, 14};
    static const int ks_b[3] = {1, 2, 3};
    static const int mg_d[4] = {4, 5, 7, 9};
    static const int mg_f[3] = {4, 7, 9};
    int rc;
    if (M::KPL == 8) rc = plan_opp<M>(ctx, mg_f, 3, ks_b, 3, pp);
    else if (std::is_same<typename M::A, double>::value) rc = plan_opp<M>(ctx, mg_d, 4, ks_d, 5, pp);
    else rc = plan_opp<M>(ctx, mg_f, 3, ks_f, 3, pp);
    pok = rc == SBCI_OK;
  }
  if (ctx->opp_form == SBCI_OPP_PAIR) {
    if (!pok) return set_error(SBCI_EINVAL, "opposite-spin sigma: the pair form does not fit in LDS");
    form = SBCI_OPP_PAIR;
    return SBCI_OK;
  }
  if (ctx->opp_form == SBCI_OPP_ORBITAL || ctx->opp_form == SBCI_OPP_ORBITAL_WINDOWED) {
    if (!qok) return set_error(SBCI_EINVAL, "opposite-spin sigma: the orbital form does not fit");
    form = SBCI_OPP_ORBITAL;
    return SBCI_OK;
  }
  if (!pok && !qok)
    return set_error(SBCI_EINVAL, "opposite-spin sigma: beta string count too large for LDS");
  if (!qok) { form = SBCI_OPP_PAIR; return SBCI_OK; }
  if (!pok) { form = SBCI_OPP_ORBITAL; return SBCI_OK; }
  const double tiles_pair = (double)pp.ngroups * pp.MG * ((B.ns + 15) / 16) * (pp.nkc * pp.KS);
  const double tiles_q =
      (double)ctx->norb * B.mt * (B.nq_pad / 16) * (pq.nkc * pq.KS) * (double)pq.nwin;
  form = 3.0 * tiles_q <= 2.0 * tiles_pair ? SBCI_OPP_ORBITAL : SBCI_OPP_PAIR;
  return SBCI_OK;
}

template <typename M, typename T>
int launch_opp(sbci_ctx *ctx, const T *c, T *out, int nvec, const __bf16 *cb = nullptr,
               int64_t ldcb = 0, double *rmax_fixed = nullptr) {
  const SpinTables &A = ctx->A, &B = ctx->B;
  if (A.s == 0 || B.m == 0) return SBCI_OK;
  if (ctx->ndet >= ((int64_t)1 << 31))
    return set_error(SBCI_EINVAL, "opposite-spin sigma: N_det must be below 2^31");
  int form = 0;
  OppPlan pp{};
  OppQPlan pq{};
  SBCI_TRY(choose_opp<M>(ctx, form, pp, pq));
  double *rmax = rmax_fixed;
  if constexpr (std::is_same<M, MF64>::value) {
    if (!rmax) {
      SBCI_TRY(ensure(ctx->ws_rmax, sizeof(double) * (size_t)A.ns * nvec));
      rmax = static_cast<double *>(ctx->ws_rmax.ptr);
    }
  }
  if (form == SBCI_OPP_ORBITAL) return launch_opp_q<M, T>(ctx, pq, c, out, nvec, rmax);
  if constexpr (std::is_same<M, MBF16>::value) {
    if (cb) {
      if ((uint64_t)A.ns * (uint64_t)ldcb >= (1ull << 32))
        return set_error(SBCI_EINVAL, "opposite-spin sigma: BF16 copy too large for 32-bit offsets");
      return launch_opp_pair<M, T, __bf16>(ctx, pp, cb, ldcb, out, nvec, nullptr);
    }
  }
  return launch_opp_pair<M, T, T>(ctx, pp, c, B.ns, out, nvec, rmax);
}

// Same-spin part with the source stripe in LDS: one workgroup per (column
// stripe of WC columns, block of list rows).  The stripe holds all R source
// rows (R * 32 bytes), so each list entry costs one 32-byte LDS read instead
// of a row-segment read from L2, and each list is read once per stripe with
// coalesced loads from the transposed lists ([entry][row]).  Work items are
// numbered row-block-major and dealt to the XCDs in contiguous ranges, so
// the workgroups of one XCD sweep the same list rows together.
template <typename T, typename V, int WC>
__global__ __launch_bounds__(1024) void k_same_lds(
    const int32_t *__restrict__ colT, const V *__restrict__ valT, int nf, int64_t R, int64_t C,
    const T *__restrict__ src, T *__restrict__ dst, int64_t nstripes, int64_t rlen,
    int64_t per_xcd, int64_t total) {
  // Row j of the stripe is 32 bytes = two 16-byte halves; rows with bit 3 of
  // j set store their halves swapped, so that the first-half reads of 64
  // random rows spread over all 64 LDS banks instead of half of them.
  constexpr int HW = WC / 2;  // elements per half
  extern __shared__ __align__(16) unsigned char smem[];
  T *L = reinterpret_cast<T *>(smem);  // [R][WC], halves swizzled
  const int64_t b = blockIdx.x;
  const int64_t w = (b & 7) * per_xcd + (b >> 3);
  if (w >= total) return;
  const int64_t rb = w / nstripes, stripe = w - rb * nstripes;
  const int64_t vo = (int64_t)blockIdx.z * R * C;
  const int64_t c0 = stripe * WC;
  for (int64_t e = threadIdx.x; e < R * WC; e += blockDim.x) {
    const int64_t j = e / WC;
    const int u = (int)(e - j * WC);
    const int pos = u ^ ((int)((j >> 3) & 1) * HW);
    L[j * WC + pos] = c0 + u < C ? src[vo + j * C + c0 + u] : (T)0;
  }
  __syncthreads();
  const int64_t r0 = rb * rlen, r1 = r0 + rlen < R ? r0 + rlen : R;
  constexpr int UN = sizeof(T) == 8 ? 4 : 8;  // list entries fetched ahead
  for (int64_t I = r0 + threadIdx.x; I < r1; I += blockDim.x) {
    T acc[WC];
#pragma unroll
    for (int u = 0; u < WC; ++u) acc[u] = 0;
    auto apply = [&](int j, T v) {
      const int sw = (j >> 3) & 1;
      const T *row = L + (int64_t)j * WC;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const T *half = row + (h ^ sw) * HW;
#pragma unroll
        for (int u = 0; u < HW; ++u) acc[h * HW + u] += v * half[u];
      }
    };
    int f = 0;
    for (; f + UN <= nf; f += UN) {
      int j[UN];
      T v[UN];
#pragma unroll
      for (int k = 0; k < UN; ++k) {
        j[k] = colT[(int64_t)(f + k) * R + I];
        v[k] = (T)valT[(int64_t)(f + k) * R + I];
      }
#pragma unroll
      for (int k = 0; k < UN; ++k) apply(j[k], v[k]);
    }
    for (; f < nf; ++f) apply(colT[(int64_t)f * R + I], (T)valT[(int64_t)f * R + I]);
    T *d = dst + vo + I * C + c0;
#pragma unroll
    for (int u = 0; u < WC; ++u)
      if (c0 + u < C) d[u] = acc[u];
  }
}

template <typename T, typename V>
int launch_same_lds(sbci_ctx *ctx, const SpinTables &S, const V *fvalT, int64_t R, int64_t C,
                    const T *src, T *dst, int nvec) {
  constexpr int WC = 32 / sizeof(T);
  const size_t lds = sizeof(T) * (size_t)R * WC;
  static bool attr = false;
  if (!attr) {
    SBCI_HIP(hipFuncSetAttribute((const void *)k_same_lds<T, V, WC>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)(120 * 1024)));
    attr = true;
  }
  const int64_t nstripes = (C + WC - 1) / WC;
  // enough workgroups for several per CU, each with >= 1024 rows of work
  int64_t rblocks = (1024 + nstripes - 1) / nstripes;
  const int64_t rmax = (R + 1023) / 1024;
  if (rblocks > rmax) rblocks = rmax;
  if (rblocks < 1) rblocks = 1;
  const int64_t rlen = (R + rblocks - 1) / rblocks;
  const int64_t total = rblocks * nstripes;
  const int64_t per_xcd = (total + 7) / 8;
  dim3 grid((unsigned)(per_xcd * 8), 1, (unsigned)nvec);
  k_same_lds<T, V, WC><<<grid, 1024, lds, ctx->stream>>>(S.fcolT, fvalT, S.nf, R, C, src, dst,
                                                        nstripes, rlen, per_xcd, total);
  SBCI_CHECK_LAUNCH();
  return SBCI_OK;
}

// Same-spin part above the LDS-stripe range: the stripe of 64-byte source
// rows (8 FP64 or 16 FP32 columns) no longer fits in LDS whole, so it passes
// through LDS in blocks of rb rows.  One workgroup (16 waves) per (row panel,
// stripe); wave w owns the 64-row groups w, w + 16, ... of its panel (RPT of
// them, lane = row) and keeps their WC accumulators in registers across the
// blocks.  For each block the workgroup stages the block's stripe, then each
// wave walks its groups' block-binned lists: one 2-byte block-local column
// and one value per lane per slot, coalesced, and four 16-byte LDS reads.
// Rows sit 80 bytes apart (four 16-byte chunks and one of padding), so the
// chunks that 16 lanes read from random rows spread over all LDS banks, and
// the four reads of a row take one address with immediate offsets.  An XOR
// swizzle of the chunks spread the banks as well but cost about 10 VALU
// instructions per slot in address arithmetic (25 % of the FP64 kernel).
// Work items are numbered
// row-panel-major and dealt to the XCDs in contiguous ranges: the workgroups
// of one XCD sweep the same panel's lists together.
template <typename T, typename V, int RPT>
__global__ __launch_bounds__(1024) void k_same_blk(
    const uint16_t *__restrict__ bcol, const V *__restrict__ bval, const int32_t *__restrict__ boff,
    int nblk, int rb, int64_t R, int64_t C, const T *__restrict__ src, T *__restrict__ dst,
    int64_t nstripes, int64_t ngrp, int64_t per_xcd, int64_t total) {
  constexpr int WC = 64 / sizeof(T);   // columns of a stripe
  constexpr int CE = 16 / sizeof(T);   // elements of a 16-byte chunk
  constexpr int NW = 16;               // waves per workgroup
  using T16 = typename std::conditional<sizeof(T) == 8, double2, float4>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  T16 *L = reinterpret_cast<T16 *>(smem);  // [rb][5] chunks (the fifth is padding)
  const int64_t b = blockIdx.x;
  const int64_t w = (b & 7) * per_xcd + (b >> 3);
  if (w >= total) return;
  const int64_t panel = w / nstripes, stripe = w - panel * nstripes;
  const int64_t vo = (int64_t)blockIdx.z * R * C;
  const int64_t c0 = stripe * WC;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t g0 = panel * NW * RPT;
  T acc[RPT][WC];
#pragma unroll
  for (int k = 0; k < RPT; ++k)
#pragma unroll
    for (int u = 0; u < WC; ++u) acc[k][u] = 0;
  const bool full = c0 + WC <= C;
  for (int blk = 0; blk < nblk; ++blk) {
    const int64_t j0 = (int64_t)blk * rb;
    const int rows = (int)(R - j0 < rb ? R - j0 : rb);
    __syncthreads();  // the previous block's readers are done
    for (int e = threadIdx.x; e < rows * 4; e += 1024) {
      const int j = e >> 2, q = e & 3;
      const T *g = src + vo + (j0 + j) * C + c0 + q * CE;
      T16 v;
      T *pv = reinterpret_cast<T *>(&v);
      if (full) {
#pragma unroll
        for (int u = 0; u < CE; ++u) pv[u] = g[u];
      } else {
#pragma unroll
        for (int u = 0; u < CE; ++u) pv[u] = c0 + q * CE + u < C ? g[u] : (T)0;
      }
      L[j * 5 + q] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int64_t grp = g0 + wave + NW * k;
      if (grp < ngrp) {
        const int s0 = boff[grp * nblk + blk], s1 = boff[grp * nblk + blk + 1];
        auto apply = [&](int j, T v) {
          const T16 *Lj = L + j * 5;  // one address; the chunks are immediate offsets
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const T16 x = Lj[q];
            const T *px = reinterpret_cast<const T *>(&x);
#pragma unroll
            for (int u = 0; u < CE; ++u) acc[k][q * CE + u] += v * px[u];
          }
        };
        constexpr int UN = sizeof(T) == 8 ? 4 : 8;
        int sl = s0;
        for (; sl + UN <= s1; sl += UN) {
          int j[UN];
          T v[UN];
#pragma unroll
          for (int i = 0; i < UN; ++i) {
            j[i] = bcol[(int64_t)(sl + i) * 64 + lane];
            v[i] = (T)bval[(int64_t)(sl + i) * 64 + lane];
          }
#pragma unroll
          for (int i = 0; i < UN; ++i) apply(j[i], v[i]);
        }
        for (; sl < s1; ++sl) apply(bcol[(int64_t)sl * 64 + lane], (T)bval[(int64_t)sl * 64 + lane]);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int64_t I = (g0 + wave + NW * k) * 64 + lane;
    if (I < R) {
      T *d = dst + vo + I * C + c0;
#pragma unroll
      for (int u = 0; u < WC; ++u)
        if (c0 + u < C) d[u] = acc[k][u];
    }
  }
}

template <typename T, typename V>
int launch_same_blk(sbci_ctx *ctx, const SpinTables &S, const V *bval, int64_t R, int64_t C,
                    const T *src, T *dst, int nvec) {
  constexpr int RPT = 4, NW = 16, WC = 64 / sizeof(T);
  const size_t lds = (size_t)kSameBlkRows * 80;
  static bool attr = false;
  if (!attr) {
    SBCI_HIP(hipFuncSetAttribute((const void *)k_same_blk<T, V, RPT>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr = true;
  }
  const int64_t nstripes = (C + WC - 1) / WC;
  const int64_t rows_per_panel = (int64_t)NW * RPT * 64;
  const int64_t npanels = (R + rows_per_panel - 1) / rows_per_panel;
  const int64_t total = npanels * nstripes;
  const int64_t per_xcd = (total + 7) / 8;
  if (per_xcd * 8 >= ((int64_t)1 << 31)) return set_error(SBCI_EINVAL, "same-spin sigma: grid too large");
  dim3 grid((unsigned)(per_xcd * 8), 1, (unsigned)nvec);
  k_same_blk<T, V, RPT><<<grid, 1024, lds, ctx->stream>>>(S.bcol, bval, S.boff, S.nblk,
                                                         kSameBlkRows, R, C, src, dst, nstripes,
                                                         S.ngrp, per_xcd, total);
  SBCI_CHECK_LAUNCH();
  return SBCI_OK;
}

template <typename T, typename V, int VC>
void launch_same_vc(sbci_ctx *ctx, const SpinTables &S, const V *fval, int64_t R, int64_t C,
                    const T *src, T *dst, int nvec, int accumulate) {
  constexpr int WAVES = 4;
  const int64_t rgroups = (R + WAVES - 1) / WAVES;
  const int64_t ctiles = (C + 64 * VC - 1) / (64 * VC);
  const int64_t total = rgroups * ctiles;
  const int64_t per_xcd = (total + 7) / 8;
  dim3 grid((unsigned)(per_xcd * 8), 1, (unsigned)nvec);
  k_same<T, V, WAVES, VC><<<grid, 64 * WAVES, 0, ctx->stream>>>(S.fcol, fval, S.nf, R, C, src, dst,
                                                               accumulate, rgroups, per_xcd, total);
}

template <typename T, typename V>
int launch_same(sbci_ctx *ctx, const SpinTables &S, const V *fval, int64_t R, int64_t C,
                const T *src, T *dst, int nvec, int accumulate) {
  if (!accumulate && S.fcolT && R >= kSameLdsMinRows && R <= kSameLdsMaxRows) {
    if constexpr (std::is_same<V, double>::value)
      return launch_same_lds<T, V>(ctx, S, S.fvalT64, R, C, src, dst, nvec);
    else
      return launch_same_lds<T, V>(ctx, S, S.fvalT32, R, C, src, dst, nvec);
  }
  if (!accumulate && S.bcol && R > kSameLdsMaxRows && R == S.ns) {
    if constexpr (std::is_same<V, double>::value)
      return launch_same_blk<T, V>(ctx, S, S.bval64, R, C, src, dst, nvec);
    else
      return launch_same_blk<T, V>(ctx, S, S.bval32, R, C, src, dst, nvec);
  }
  // widest column tile whose source rows (R x 64 VC elements) stay within
  // about half of one XCD's 4 MB L2
  const double tile1 = (double)R * 64 * sizeof(T);
  const double budget = 2.0 * 1024 * 1024;
  if (C >= 256 && 4 * tile1 <= budget)
    launch_same_vc<T, V, 4>(ctx, S, fval, R, C, src, dst, nvec, accumulate);
  else if (C >= 128 && 2 * tile1 <= budget)
    launch_same_vc<T, V, 2>(ctx, S, fval, R, C, src, dst, nvec, accumulate);
  else
    launch_same_vc<T, V, 1>(ctx, S, fval, R, C, src, dst, nvec, accumulate);
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

// Optional per-part timing: ev[0..5] recorded on the launch stream around
// the five parts (alpha lists, opposite spin, transpose, beta lists, add).
struct PartEvents {
  hipEvent_t ev[6];
};

int rec(sbci_ctx *ctx, PartEvents *pe, int i) {
  if (pe) SBCI_HIP(hipEventRecord(pe->ev[i], ctx->stream));
  return SBCI_OK;
}

// Row r of the dense same-spin operator: zeros, then the list entries
// (one workgroup per row; a kernel, not a memset, so that a captured sigma
// records no memset node).
template <typename V>
__global__ void k_densify(const int32_t *__restrict__ fcol, const V *__restrict__ fval, int nf,
                          int64_t ns, V *__restrict__ H) {
  const int64_t r = blockIdx.x;
  V *row = H + r * ns;
  for (int64_t j = threadIdx.x; j < ns; j += blockDim.x) row[j] = (V)0;
  __syncthreads();
  for (int e = threadIdx.x; e < nf; e += blockDim.x) row[fcol[r * nf + e]] = fval[r * nf + e];
}

// Row r of the BF16 operator without its diagonal, and the diagonal in FP32.
__global__ void k_densify_bf16(const int32_t *__restrict__ fcol, const float *__restrict__ fval,
                               int nf, int64_t ns, int64_t ld, __hip_bfloat16 *__restrict__ H,
                               float *__restrict__ dd) {
  const int64_t r = blockIdx.x;
  __hip_bfloat16 *row = H + r * ld;
  for (int64_t j = threadIdx.x; j < ld; j += blockDim.x) row[j] = __float2bfloat16(0.0f);
  __syncthreads();
  for (int e = threadIdx.x; e < nf; e += blockDim.x) {
    const int32_t c = fcol[r * nf + e];
    if (c == r) dd[r] = fval[r * nf + e];
    else row[c] = __float2bfloat16(fval[r * nf + e]);
  }
}

// The BF16 sigma's same-spin part: the dense BF16 product wherever the
// dense operator fits (kDenseMaxRows), from the LDS-stripe range up (below
// it the lists are already fast); SBCI_SAME_LISTS / _DENSE force it.
bool use_dense_bf16(const sbci_ctx *ctx, const SpinTables &S) {
  if (ctx->same_form == SBCI_SAME_DENSE) return true;
  if (ctx->same_form == SBCI_SAME_LISTS) return false;
  return S.ns >= kSameLdsMinRows && S.ns <= kDenseMaxRows;
}

int dense_same_bf16(sbci_ctx *ctx, SpinTables &S, const __hip_bfloat16 **H, const float **dd) {
  SpinTables &O = S.shared ? ctx->A : S;
  if (O.ns > kDenseMaxRows)
    return set_error(SBCI_EINVAL, "same-spin sigma: too many strings for the dense form");
  if (!O.hdbf) {
    const int64_t ld = (O.ns + 63) / 64 * 64;  // rows padded with zeros (whole K panels)
    SBCI_HIP(hipMalloc(&O.hdbf, sizeof(__hip_bfloat16) * (size_t)O.ns * ld));
    SBCI_HIP(hipMalloc(&O.hdd32, sizeof(float) * (size_t)O.ns));
    k_densify_bf16<<<(unsigned)O.ns, 256, 0, ctx->stream>>>(O.fcol, O.fval32, O.nf, O.ns, ld,
                                                            O.hdbf, O.hdd32);
    SBCI_CHECK_LAUNCH();
  }
  if (&O != &S) {
    S.hdbf = O.hdbf;
    S.hdd32 = O.hdd32;
  }
  *H = O.hdbf;
  *dd = O.hdd32;
  return SBCI_OK;
}

// BF16 same-spin products of the BF16 sigma: alpha (side 0) writes
// out = H_alpha C from C^T in BF16, beta (side 1) adds C H_beta from C in
// BF16; H is [ns][ldh] with ldh = ns rounded up to 64 (zero padded).
int64_t pad64(int64_t x) { return (x + 63) / 64 * 64; }

// The vector's BF16 copy for one side's product, rows zero padded to 64:
// alpha takes C^T [nb][pad(na)], beta C [na][pad(nb)] (which also feeds the
// gathers of the opposite-spin pair form).  It lives in ws_t until the next
// copy replaces it.
int bf16_copy(sbci_ctx *ctx, int side, const float *c, int nvec, const __bf16 **cb) {
  const int64_t na = ctx->A.ns, nb = ctx->B.ns;
  const int64_t Kp = pad64(side == 0 ? na : nb), rows = side == 0 ? nb : na;
  SBCI_TRY(ensure(ctx->ws_t, sizeof(__bf16) * (size_t)rows * Kp * nvec));
  __bf16 *d = static_cast<__bf16 *>(ctx->ws_t.ptr);
  if (side == 0) {
    const dim3 gt((unsigned)((nb + TT - 1) / TT), (unsigned)((Kp + TT - 1) / TT), (unsigned)nvec);
    k_to_bf16<true><<<gt, dim3(TT, 8), 0, ctx->stream>>>(c, d, na, nb, Kp);
  } else {
    const dim3 gt((unsigned)((Kp + TT - 1) / TT), (unsigned)((na + TT - 1) / TT), (unsigned)nvec);
    k_to_bf16<false><<<gt, dim3(TT, 8), 0, ctx->stream>>>(c, d, na, nb, Kp);
  }
  SBCI_CHECK_LAUNCH();
  *cb = d;
  return SBCI_OK;
}

// The product on the copy cb that bf16_copy made for the same side.
int launch_gemm_bf16(sbci_ctx *ctx, int side, const float *c, const __bf16 *cb,
                     const __hip_bfloat16 *H, const float *dd, float *out, int nvec) {
  const int64_t na = ctx->A.ns, nb = ctx->B.ns, nd = ctx->ndet;
  const int64_t Kp = pad64(side == 0 ? na : nb);
  const int64_t tm = (na + 127) / 128, tn = (nb + 255) / 256;
  const int64_t total = tm * tn, per_xcd = (total + 7) / 8;
  if (per_xcd * 8 >= ((int64_t)1 << 31)) return set_error(SBCI_EINVAL, "same-spin sigma: grid too large");
  const dim3 grid((unsigned)(per_xcd * 8), (unsigned)nvec);
  const __bf16 *Hb = reinterpret_cast<const __bf16 *>(H);
  if (side == 0)
    k_gemm_bf16<0><<<grid, 512, 0, ctx->stream>>>(na, nb, Kp, Hb, Kp, 0, cb, Kp, nb * Kp, c, nd, dd,
                                                  out, nb, nd, 0, tn, per_xcd, total);
  else
    k_gemm_bf16<1><<<grid, 512, 0, ctx->stream>>>(na, nb, Kp, cb, Kp, na * Kp, Hb, Kp, 0, c, nd, dd,
                                                  out, nb, nd, 1, tn, per_xcd, total);
  SBCI_CHECK_LAUNCH();
  return SBCI_OK;
}

bool use_dense(const sbci_ctx *ctx, const SpinTables &S) {
  if (ctx->same_form == SBCI_SAME_DENSE) return true;
  if (ctx->same_form == SBCI_SAME_LISTS) return false;
  return S.ns > kSameLdsMaxRows && S.ns <= kDenseMaxRows && (int64_t)S.nf * 10 >= S.ns;
}

// The dense operator of a spin in the precision of T, built on first use
// from the lists (beta uses alpha's when the two spins share tables).
template <typename T>
int dense_same(sbci_ctx *ctx, SpinTables &S, const T **out) {
  SpinTables &O = S.shared ? ctx->A : S;
  if (O.ns > kDenseMaxRows)
    return set_error(SBCI_EINVAL, "same-spin sigma: too many strings for the dense form");
  T **slot;
  const T *vals;
  if constexpr (std::is_same<T, double>::value) {
    slot = &O.hd64;
    vals = O.fval64;
  } else {
    slot = &O.hd32;
    vals = O.fval32;
  }
  if (!*slot) {
    const size_t bytes = sizeof(T) * (size_t)O.ns * O.ns;
    SBCI_HIP(hipMalloc(slot, bytes));
    k_densify<T><<<(unsigned)O.ns, 256, 0, ctx->stream>>>(O.fcol, vals, O.nf, O.ns, *slot);
    SBCI_CHECK_LAUNCH();
  }
  if (&O != &S) {
    if constexpr (std::is_same<T, double>::value) S.hd64 = O.hd64; else S.hd32 = O.hd32;
  }
  *out = *slot;
  return SBCI_OK;
}

// The block-binned lists of a spin above the LDS-stripe range, built on
// first use (in the owner of shared tables).  Without permission to
// allocate, a spin whose lists are not built yet keeps the L2-streaming
// kernel.
int prepare_blk(sbci_ctx *ctx, SpinTables &S, bool may_alloc) {
  SpinTables &O = S.shared ? ctx->A : S;
  if (O.ns <= kSameLdsMaxRows || O.nf < 1) return SBCI_OK;
  if (!O.bcol) {
    if (!may_alloc) return SBCI_OK;
    SBCI_TRY(build_blk_lists(ctx, O));
  }
  if (&O != &S) {
    S.nblk = O.nblk;
    S.ngrp = O.ngrp;
    S.boff = O.boff;
    S.bcol = O.bcol;
    S.bval64 = O.bval64;
    S.bval32 = O.bval32;
  }
  return SBCI_OK;
}

template <typename T>
int launch_gemm(sbci_ctx *ctx, int64_t Mr, int64_t N, int64_t K, const T *A, int64_t lda,
                int64_t sA, const T *B, int64_t ldb, int64_t sB, T *out, int64_t ldc, int64_t sC,
                int nvec, int accumulate) {
  // tile shapes measured on gfx950 at 14190^3: FP64 128 x 256 (8 waves,
  // 48 TF/s; 16 waves spill the accumulators), FP32 256 x 256 (16 waves,
  // 97 TF/s); both about 1.4x the 128 x 128 tile
  using G = typename std::conditional<std::is_same<T, double>::value, MF64, MF32>::type;
  constexpr int WM = std::is_same<T, double>::value ? 2 : 4, WN = 4;
  const int64_t tm = (Mr + 64 * WM - 1) / (64 * WM), tn = (N + 64 * WN - 1) / (64 * WN);
  const int64_t total = tm * tn, per_xcd = (total + 7) / 8;
  if (per_xcd * 8 >= ((int64_t)1 << 31)) return set_error(SBCI_EINVAL, "same-spin sigma: grid too large");
  k_gemm<G, T, WM, WN><<<dim3((unsigned)(per_xcd * 8), (unsigned)nvec), 64 * WM * WN, 0, ctx->stream>>>(
      Mr, N, K, A, lda, sA, B, ldb, sB, out, ldc, sC, accumulate, tn, per_xcd, total);
  SBCI_CHECK_LAUNCH();
  return SBCI_OK;
}

// ct_fixed / st_fixed: caller-provided scratch for the beta part's transposed
// operand and result (each nvec * ndet elements); nullptr takes the
// context's workspaces, allocated on first use.
template <typename T, typename M>
int sigma_t(sbci_ctx *ctx, const T *c, T *out, int nvec, PartEvents *pe = nullptr,
            T *ct_fixed = nullptr, T *st_fixed = nullptr, double *rmax_fixed = nullptr) {
  SpinTables &A = ctx->A, &B = ctx->B;
  const int64_t na = A.ns, nb = B.ns, nd = ctx->ndet;
  const bool dbl = std::is_same<T, double>::value;
  constexpr bool bf = std::is_same<M, MBF16>::value;
  const bool bfA = bf && use_dense_bf16(ctx, A), bfB = bf && use_dense_bf16(ctx, B);
  const bool denseA = !bfA && use_dense(ctx, A), denseB = !bfB && use_dense(ctx, B);
  const bool may_alloc = !ct_fixed;
  if (!bfA && !denseA) SBCI_TRY(prepare_blk(ctx, A, may_alloc));
  if (!bfB && !denseB) SBCI_TRY(prepare_blk(ctx, B, may_alloc));
  // alpha part (plain write), then opposite-spin (accumulate)
  SBCI_TRY(rec(ctx, pe, 0));
  if constexpr (bf) {
    if (bfA) {
      const __hip_bfloat16 *H = nullptr;
      const float *dd = nullptr;
      const __bf16 *ct = nullptr;
      SBCI_TRY(dense_same_bf16(ctx, A, &H, &dd));
      SBCI_TRY(bf16_copy(ctx, 0, c, nvec, &ct));
      SBCI_TRY(launch_gemm_bf16(ctx, 0, c, ct, H, dd, out, nvec));
    }
  }
  if (bfA) {
  } else if (denseA) {
    const T *H = nullptr;
    SBCI_TRY(dense_same<T>(ctx, A, &H));
    SBCI_TRY(launch_gemm<T>(ctx, na, nb, na, H, na, 0, c, nb, nd, out, nb, nd, nvec, 0));
  } else if (dbl) {
    SBCI_TRY((launch_same<T, double>(ctx, A, A.fval64, na, nb, c, out, nvec, 0)));
  } else {
    SBCI_TRY((launch_same<T, float>(ctx, A, A.fval32, na, nb, c, out, nvec, 0)));
  }
  // the BF16 copy of C that the beta product needs is made here, before the
  // opposite-spin part, whose pair form then gathers from it (half the bytes
  // of the FP32 vector, and the values it rounds them to anyway); its time
  // is counted with the alpha part
  const __bf16 *cbeta = nullptr;
  if constexpr (bf) {
    if (bfB) SBCI_TRY(bf16_copy(ctx, 1, c, nvec, &cbeta));
  }
  SBCI_TRY(rec(ctx, pe, 1));
  SBCI_TRY((launch_opp<M, T>(ctx, c, out, nvec, cbeta, cbeta ? pad64(nb) : 0, rmax_fixed)));
  SBCI_TRY(rec(ctx, pe, 2));
  if constexpr (bf) {
    if (bfB) {
      // beta part as C H_beta on BF16 MFMA, accumulated in place
      const __hip_bfloat16 *H = nullptr;
      const float *dd = nullptr;
      SBCI_TRY(dense_same_bf16(ctx, B, &H, &dd));
      SBCI_TRY(rec(ctx, pe, 3));
      SBCI_TRY(launch_gemm_bf16(ctx, 1, c, cbeta, H, dd, out, nvec));
      SBCI_TRY(rec(ctx, pe, 4));
      SBCI_TRY(rec(ctx, pe, 5));
      return SBCI_OK;
    }
  }
  if (denseB) {
    // beta part as C H_beta, accumulated in place (no transposes)
    const T *H = nullptr;
    SBCI_TRY(dense_same<T>(ctx, B, &H));
    SBCI_TRY(rec(ctx, pe, 3));
    SBCI_TRY(launch_gemm<T>(ctx, na, nb, nb, c, nb, nd, H, nb, 0, out, nb, nd, nvec, 1));
    SBCI_TRY(rec(ctx, pe, 4));
    SBCI_TRY(rec(ctx, pe, 5));
    return SBCI_OK;
  }
  // beta part on C^T, added back transposed
  T *ct = ct_fixed, *st = st_fixed;
  if (!ct || !st) {
    const size_t vbytes = sizeof(T) * (size_t)nd * nvec;
    SBCI_TRY(ensure(ctx->ws_t, vbytes));
    SBCI_TRY(ensure(ctx->ws_s, vbytes));
    ct = static_cast<T *>(ctx->ws_t.ptr);
    st = static_cast<T *>(ctx->ws_s.ptr);
  }
  SBCI_TRY(launch_transpose<T>(ctx, c, ct, na, nb, nvec, false));
  SBCI_TRY(rec(ctx, pe, 3));
  if (dbl)
    SBCI_TRY((launch_same<T, double>(ctx, B, B.fval64, nb, na, ct, st, nvec, 0)));
  else
    SBCI_TRY((launch_same<T, float>(ctx, B, B.fval32, nb, na, ct, st, nvec, 0)));
  SBCI_TRY(rec(ctx, pe, 4));
  SBCI_TRY(launch_transpose<T>(ctx, st, out, nb, na, nvec, true));
  SBCI_TRY(rec(ctx, pe, 5));
  return SBCI_OK;
}

}  // namespace

namespace {
int sigma_dispatch(sbci_ctx *ctx, const void *c, void *out, int nvec, int mode, PartEvents *pe) {
  if (ctx->sym) return sigma_sym(ctx, c, out, nvec, mode, pe ? pe->ev : nullptr);
  switch (mode) {
    case SBCI_F64:
      return sigma_t<double, MF64>(ctx, static_cast<const double *>(c), static_cast<double *>(out),
                                   nvec, pe);
    case SBCI_F32:
      return sigma_t<float, MF32>(ctx, static_cast<const float *>(c), static_cast<float *>(out),
                                  nvec, pe);
    case SBCI_BF16:
      return sigma_t<float, MBF16>(ctx, static_cast<const float *>(c), static_cast<float *>(out),
                                   nvec, pe);
    default:
      return set_error(SBCI_EINVAL, "unknown sigma dtype");
  }
}
}  // namespace

int sigma(sbci_ctx *ctx, const void *c, void *out, int nvec, int mode) {
  return sigma_dispatch(ctx, c, out, nvec, mode, nullptr);
}

}  // namespace sbci

// Scratch of the allocation-free sigma: the beta part's transposed operand
// and result.  Each device that loads the library holds one copy until the
// process ends; host code reaches it only through the address that
// hipGetSymbolAddress returns for that device.
static __device__ __align__(256) unsigned char scratch[sbci::kNoAllocScratchBytes];

namespace sbci {

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, looked up once per device with
// that device current.
int scratch_address(int device, void **out) {
  if (device < 0 || device >= kMaxDevices)
    return set_error(SBCI_EDEVICE, "allocation-free sigma: device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = 0;
    SBCI_HIP(hipGetDevice(&cur));
    if (cur != device) SBCI_HIP(hipSetDevice(device));
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) SBCI_HIP(hipSetDevice(cur));
    if (e != hipSuccess || !p)
      return set_error(SBCI_EDEVICE, std::string("allocation-free sigma: hipGetSymbolAddress: ") +
                                         hipGetErrorString(e));
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return SBCI_OK;
}
}  // namespace

int sigma_noalloc(sbci_ctx *ctx, const void *c, void *out, int nvec, int mode) {
  if (ctx->sym)
    return set_error(SBCI_EINVAL, "allocation-free sigma: symmetry-blocked contexts are not supported");
  if (mode != SBCI_F64 && mode != SBCI_F32)
    return set_error(SBCI_EINVAL, "allocation-free sigma: FP64 or FP32 only (the BF16 form builds "
                                  "its operand copies on first use)");
  if (use_dense(ctx, ctx->A) || use_dense(ctx, ctx->B))
    return set_error(SBCI_EINVAL, "allocation-free sigma: the dense same-spin form is not "
                                  "supported (its operator is built on first use)");
  int form = 0;
  SBCI_TRY(opp_form(ctx, mode, &form));
  if (form != SBCI_OPP_PAIR)
    return set_error(SBCI_EINVAL, "allocation-free sigma: only the pair opposite-spin form is "
                                  "supported (the orbital form stages a copy of c)");
  const size_t es = mode == SBCI_F64 ? 8 : 4;
  const size_t half = (es * (size_t)ctx->ndet * (size_t)nvec + 255) / 256 * 256;
  const size_t rtail = mode == SBCI_F64 ? (8 * (size_t)ctx->A.ns * (size_t)nvec + 255) / 256 * 256 : 0;
  if (2 * half + rtail > kNoAllocScratchBytes)
    return set_error(SBCI_EINVAL, "allocation-free sigma: needs two operands of nvec * ndet "
                                  "elements (and, in FP64, nvec * N_alpha row maxima) within the "
                                  "64 MiB scratch");
  void *p = nullptr;
  SBCI_TRY(scratch_address(ctx->device, &p));
  unsigned char *base = static_cast<unsigned char *>(p);
  if (mode == SBCI_F64)
    return sigma_t<double, MF64>(ctx, static_cast<const double *>(c), static_cast<double *>(out),
                                 nvec, nullptr, reinterpret_cast<double *>(base),
                                 reinterpret_cast<double *>(base + half),
                                 reinterpret_cast<double *>(base + 2 * half));
  return sigma_t<float, MF32>(ctx, static_cast<const float *>(c), static_cast<float *>(out), nvec,
                              nullptr, reinterpret_cast<float *>(base),
                              reinterpret_cast<float *>(base + half));
}

int same_lists_block(sbci_ctx *ctx, const int32_t *fcol, const void *fval, int nf, int64_t R,
                     int64_t C, const void *src, void *dst, int mode) {
  SpinTables P{};
  P.fcol = const_cast<int32_t *>(fcol);
  P.nf = nf;
  if (mode == SBCI_F64)
    return launch_same<double, double>(ctx, P, static_cast<const double *>(fval), R, C,
                                       static_cast<const double *>(src), static_cast<double *>(dst),
                                       1, 1);
  return launch_same<float, float>(ctx, P, static_cast<const float *>(fval), R, C,
                                   static_cast<const float *>(src), static_cast<float *>(dst), 1, 1);
}

int same_form(sbci_ctx *ctx, int spin, int dtype, int *form) {
  const SpinTables &S = spin == 0 ? ctx->A : ctx->B;
  const bool dense = dtype == SBCI_BF16 ? use_dense_bf16(ctx, S) : use_dense(ctx, S);
  *form = dense ? SBCI_SAME_DENSE : SBCI_SAME_LISTS;
  return SBCI_OK;
}

int opp_form(sbci_ctx *ctx, int mode, int *form) {
  OppPlan pp{};
  OppQPlan pq{};
  switch (mode) {
    case SBCI_F64: return choose_opp<MF64>(ctx, *form, pp, pq);
    case SBCI_F32: return choose_opp<MF32>(ctx, *form, pp, pq);
    case SBCI_BF16: return choose_opp<MBF16>(ctx, *form, pp, pq);
    default: return set_error(SBCI_EINVAL, "unknown sigma dtype");
  }
}

int sigma_profile(sbci_ctx *ctx, const void *c, void *out, int nvec, int mode, float *ms) {
  PartEvents pe{};
  for (int i = 0; i < 6; ++i) SBCI_HIP(hipEventCreate(&pe.ev[i]));
  int rc = sigma_dispatch(ctx, c, out, nvec, mode, &pe);
  if (rc == SBCI_OK) {
    SBCI_HIP(hipEventSynchronize(pe.ev[5]));
    for (int i = 0; i < 5; ++i) SBCI_HIP(hipEventElapsedTime(&ms[i], pe.ev[i], pe.ev[i + 1]));
  }
  for (int i = 0; i < 6; ++i) hipEventDestroy(pe.ev[i]);
  return rc;
}

}  // namespace sbci
