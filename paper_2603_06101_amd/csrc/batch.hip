// Batching form: many independent CAS instances, each with its own roots,
// solved by SBCI1 (Algorithm 1 with Supplementary Sections S1.1-S1.5) in ONE
// persistent-kernel launch captured in a hipGraph.
//
// Design
//   * One workgroup owns one instance for the whole solve: the SBCI state
//     machine (start vectors, steps, restarts, precision hand-overs, root
//     sequencing) runs on the device, its scalars in LDS, with the 2x2 / 3x3
//     Ritz problems of ritz.h solved by one lane.  No host round trip, no
//     grid-wide barrier: workgroups never wait for each other.
//   * Workgroups take instances from an atomic queue in longest-first order
//     (or input order), so uneven sizes balance across the 256 CUs.  Every
//     workgroup leaves when the queue is exhausted; every instance ends after
//     at most max_steps steps per root.
//   * Teams: an instance whose estimated work exceeds the balanced share of
//     one workgroup runs on a team of 2-4 workgroups (the lowest block
//     indices, dispatched first and co-resident).  Each member owns a range
//     of 16-row alpha tiles: its rows of sigma and of every vector pass.
//     The members run the same state machine on the same reduced values (the
//     team sums the members' partials in member order), so they take the same
//     decisions; a barrier (agent-scope release / acquire around a counter)
//     sits in every reduction and before every sigma, whose input spans all
//     members' rows.  Every wait is bounded (one second by default): past the
//     bound the team aborts the instance with SBCI_EDEVICE.
//   * sigma inside a workgroup: the one-electron and same-spin parts as two
//     dense MFMA products C * H_beta + H_alpha * C (for norb <= 10 these
//     operators are 50-95 % dense) with LDS-staged K panels; the
//     opposite-spin part per wavefront and row as an MFMA contraction of the
//     signed ERI pair tile (in registers) with s gathered rows of C,
//     scattered through the beta pair table into the wave's LDS copy of
//     sigma's row (FP64 LDS atomics).
//   * The vector passes (fused update, deflation, dots) are the same
//     arithmetic as vec.hip with workgroup-level FP64 reductions in a fixed
//     order.
//   * Launch shape (workgroup size, workgroups per CU, queue order, K panel
//     of the same-spin products) is chosen by a measured autotuner
//     (sbci_batch_tune).
#include "internal.h"
#include "mfma.h"
#include "ritz.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <utility>
#include <vector>

struct sbci_batch;

namespace sbci {
namespace {

constexpr int BMAXR = 4;     // roots per instance
constexpr int BMAX_NORB = 10;
constexpr int BMAX_NS = 252; // strings per spin, C(10, 5)
constexpr int BMAX_S = 30;   // single excitations per string, 5 * 6
constexpr int BMAX_NP = 64;  // pair rows (55 for norb = 10), padded to 16
constexpr int NVW = 7;       // work vectors: x, X, y, Y, za, zb, Z
constexpr int BMAX_TEAM = 4; // workgroups per instance
enum { SX = 0, SXX = 1, SY = 2, SYY = 3, SZA = 4, SZB = 5, SZ = 6 };

struct BInst {
  int ns_a, ns_b, s_a, s_b, nf_a, nf_b, npair, nroots;
  int64_t ndet, ns_pad_b;
  const Ent *tab_a;
  const uint32_t *pair_b;
  const uint4 *quad_r_b, *quad_s_b;  // pair codes as per-lane quads (see internal.h)
  const double *H64_a, *H64_b;  // dense same-spin operators [ns][ns] (symmetric)
  const float *H32_a, *H32_b;
  const double *W64;
  const float *W32;
  const __bf16 *Wbf;
  const double *D64;
  const float *D32;
  double *v64;  // [NVW + nroots][ndet]
  float *v32;   // [NVW + nroots][ndet] (precision form only)
};

struct BOut {
  double E[BMAXR];
  double dz[BMAXR];
  uint64_t t0, t1;  // device real-time counter at the instance's start and end
  uint64_t tsig[2]; // counter ticks in the sigma parts: same-spin, opposite-spin
  int status, nconv, nsteps, nrestarts, nsig64, nsiglow, pad0, pad1;
};

struct BParams {
  double eps0, r0, b_th, eps1, x_th1, x_th2, r1, mix_eps0, mix_r0, bf16_eps0, bf16_r0, floor,
      lindep;
  int max_cycle, max_steps, precision, mix_stall;
  uint64_t team_wait;  // bound of a team barrier wait, real-time counter ticks
  int kp;  // K panel of the same-spin GEMMs: 8 or 16
};

// ------------------------------------------------------------ reductions
template <int NT>
struct Red {
  double w[NT / 64][16];
  double out[16];
  unsigned gen;  // team barriers passed by this member
  unsigned red;  // team reductions done (selects the partials buffer)
  int abort;     // the team gave up waiting
};

// Team state in global memory, one per team instance (zeroed by the reset
// kernel before every solve).
struct TeamSync {
  unsigned cnt;    // arrivals, monotonic over the solve
  unsigned abort;  // set by the first member that times out
  unsigned pad[62];
  double part[2][BMAX_TEAM][16];  // partial sums, double-buffered by reduction
};

// The rows a workgroup owns: all of an instance (T = 1), or member m's range
// of 16-row alpha tiles.
struct Team {
  TeamSync *ts;
  uint64_t wait;     // bound of a barrier wait (ticks)
  int T, m;
  int t0, t1;        // alpha tiles
  int a0, a1;        // alpha rows
  int64_t r0, r1;    // determinant rows
};

__device__ inline Team make_team(int nsa, int64_t nsb, TeamSync *ts, int T, int m, uint64_t wait) {
  Team t;
  t.ts = ts;
  t.wait = wait;
  t.T = T;
  t.m = m;
  const int tiles = (nsa + 15) / 16;
  t.t0 = m * tiles / T;
  t.t1 = (m + 1) * tiles / T;
  t.a0 = t.t0 * 16 < nsa ? t.t0 * 16 : nsa;
  t.a1 = t.t1 * 16 < nsa ? t.t1 * 16 : nsa;
  t.r0 = (int64_t)t.a0 * nsb;
  t.r1 = (int64_t)t.a1 * nsb;
  return t;
}

constexpr uint64_t kTeamWaitTicks = 100000000ull;  // default bound: 1 s of the 100 MHz real-time counter
constexpr uint64_t kTicksPerUs = 100;

// Team barrier: every member's prior global writes become visible to every
// member.  Each thread releases at agent scope, thread 0 arrives and waits
// (bounded) for all members, each thread acquires.  A lone workgroup only
// synchronises its threads.
template <int NT>
__device__ void team_sync(const Team &tm, Red<NT> &R) {
  if (tm.T <= 1) {
    __syncthreads();
    return;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0 && !R.abort) {
    const unsigned target = (R.gen + 1u) * (unsigned)tm.T;
    __hip_atomic_fetch_add(&tm.ts->cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    for (;;) {
      if (__hip_atomic_load(&tm.ts->cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
      if (__hip_atomic_load(&tm.ts->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
          __builtin_amdgcn_s_memrealtime() - t0 > tm.wait) {
        __hip_atomic_store(&tm.ts->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        R.abort = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    R.gen += 1u;
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// Sum v[0..q) over the workgroup, then over the team; the result lands in
// r.out (all threads read it after the trailing barrier).  Fixed order:
// lanes by xor tree, waves in index order, members in index order.
template <int NT, int Q>
__device__ void wg_sum(double (&v)[Q], int q, Red<NT> &r, const Team &tm) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    if (j < q) {
      double x = v[j];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
      if (lane == 0) r.w[wv][j] = x;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < q) {
    double s = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += r.w[w][threadIdx.x];
    r.out[threadIdx.x] = s;
  }
  __syncthreads();
  if (tm.T > 1) {
    const int buf = (int)(r.red & 1u);
    if ((int)threadIdx.x < q) tm.ts->part[buf][tm.m][threadIdx.x] = r.out[threadIdx.x];
    team_sync<NT>(tm, r);
    if ((int)threadIdx.x < q) {
      double s = 0;
      for (int mm = 0; mm < tm.T; ++mm) s += tm.ts->part[buf][mm][threadIdx.x];
      r.out[threadIdx.x] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) r.red += 1u;
    __syncthreads();
  }
}

// ------------------------------------------------------------ control state
// Ritz result as plain data (LDS variables cannot have initialisers).
struct RitzS {
  int rank_ok, coef_ok;
  double E[3], a1[3], a2[3], b, c, k;
};
__device__ inline RitzS pod(const Ritz &r) {
  RitzS o;
  o.rank_ok = r.rank_ok;
  o.coef_ok = r.coef_ok;
  for (int i = 0; i < 3; ++i) {
    o.E[i] = r.E[i];
    o.a1[i] = r.a1[i];
    o.a2[i] = r.a2[i];
  }
  o.b = r.b;
  o.c = r.c;
  o.k = r.k;
  return o;
}

struct Ctl {
  int alpha, seg, t, steps_root, phase, seg_start, stall, done, any_noconv, nconv, status;
  int m64[NVW], m32[NVW];  // logical slot -> physical vector
  int nsteps, nrestarts, nsig64, nsiglow;
  uint64_t tsig[2];
  double E, sx, bestE;
  double Ec[BMAXR];
  double h1[16], h2[4], h3[4];
  RitzS last, r;
  // scratch of the start (S1.1)
  int64_t idx[BMAXR];
  double Hs[BMAXR * BMAXR], w[BMAXR], U[BMAXR * BMAXR];
  double dzroot;
  int action;
};

// ------------------------------------------------------------ WG sigma
template <typename T>
struct DenseH;
template <>
struct DenseH<double> {
  __device__ static const double *a(const BInst &I) { return I.H64_a; }
  __device__ static const double *b(const BInst &I) { return I.H64_b; }
};
template <>
struct DenseH<float> {
  __device__ static const float *a(const BInst &I) { return I.H32_a; }
  __device__ static const float *b(const BInst &I) { return I.H32_b; }
};

// One-electron and same-spin part as two dense products on MFMA:
//   out = C * H_beta + H_alpha * C       (C is [ns_a][ns_b]; H_s symmetric)
// for the output tile rows [tr0, tr1) (16 alpha rows each).  For norb <= 10
// the same-spin operators are 50-95 % dense, so the dense form does little
// extra work and runs at matrix-core rate.  K panels of both operands are
// staged in LDS; each wavefront owns whole 16-row tile rows and a block of
// CB column tiles per pass.
template <typename T, typename M, int NT>
__device__ void wg_same_dense(const BInst &I, const T *__restrict__ c, T *__restrict__ out,
                              int kp, char *lds, int tr0, int tr1) {
  static_assert(M::KPL == 1 && M::KSTEP == 4, "dense same-spin GEMM uses 16x16x4 MFMA");
  using Frag = typename M::Frag;
  using Out = typename M::Out;
  constexpr int NW = NT / 64;
  constexpr int TMMAX = (BMAX_NS + 15) / 16;
  constexpr int RW = (TMMAX + NW - 1) / NW;          // tile rows per wave
  constexpr int CB = RW >= 8 ? 1 : 8 / RW;           // column tiles per wave and pass
  const int nsa = I.ns_a, nsb = I.ns_b;
  const int tm = tr1 - tr0, tn = (nsb + 15) / 16;  // tm <= TMMAX
  const int mp = tm * 16;
  const int row0 = tr0 * 16;
  const int lda = kp + 1, ldb = CB * 16 + 1;
  T *Ap = reinterpret_cast<T *>(lds);                 // [mp][lda]
  T *Bp = Ap + (size_t)(TMMAX * 16) * lda;            // [kp][ldb]
  const T *Ha = DenseH<T>::a(I), *Hb = DenseH<T>::b(I);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, li = lane & 15, g = lane >> 4;
  for (int n0 = 0; n0 < tn; n0 += CB) {
    Out acc[RW][CB];
#pragma unroll
    for (int u = 0; u < RW; ++u)
#pragma unroll
      for (int v = 0; v < CB; ++v) acc[u][v] = Out{0, 0, 0, 0};
    // product 0: C * H_beta (K = ns_b); product 1: H_alpha * C (K = ns_a)
    for (int prod = 0; prod < 2; ++prod) {
      const int K = prod == 0 ? nsb : nsa;
      for (int k0 = 0; k0 < K; k0 += kp) {
        // A panel: this range's rows of C (prod 0) or H_alpha (prod 1),
        // columns k0..k0+kp
        for (int e = tid; e < mp * kp; e += NT) {
          const int r = e / kp, k = e - r * kp, kk = k0 + k, rr = row0 + r;
          T v = (T)0;
          if (rr < nsa && kk < K) v = prod == 0 ? c[(int64_t)rr * nsb + kk] : Ha[(int64_t)rr * nsa + kk];
          Ap[r * lda + k] = v;
        }
        // B panel: rows k0..k0+kp of H_beta (prod 0) or C (prod 1), CB column tiles
        for (int e = tid; e < kp * CB * 16; e += NT) {
          const int k = e / (CB * 16), j = e - k * (CB * 16), kk = k0 + k, col = n0 * 16 + j;
          T v = (T)0;
          if (kk < K && col < nsb)
            v = prod == 0 ? Hb[(int64_t)kk * nsb + col] : c[(int64_t)kk * nsb + col];
          Bp[k * ldb + j] = v;
        }
        __syncthreads();
        for (int ks = 0; ks < kp / 4; ++ks) {
          Frag b[CB];
#pragma unroll
          for (int v = 0; v < CB; ++v) b[v] = Bp[(ks * 4 + g) * ldb + v * 16 + li];
#pragma unroll
          for (int u = 0; u < RW; ++u) {
            const int tr = wv + u * NW;
            if (tr < tm) {
              const Frag a = Ap[(tr * 16 + li) * lda + ks * 4 + g];
#pragma unroll
              for (int v = 0; v < CB; ++v) acc[u][v] = M::mma(a, b[v], acc[u][v]);
            }
          }
        }
        __syncthreads();
      }
    }
#pragma unroll
    for (int u = 0; u < RW; ++u) {
      const int tr = wv + u * NW;
      if (tr < tm) {
#pragma unroll
        for (int v = 0; v < CB; ++v) {
          const int col = (n0 + v) * 16 + li;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = row0 + tr * 16 + M::orow(g, r);
            if (row < nsa && col < nsb) out[(int64_t)row * nsb + col] = (T)acc[u][v][r];
          }
        }
      }
    }
  }
  __syncthreads();
}

// Team form of the same dense products.  A member owns few tile rows
// (5-8 of 16 at norb = 10), so a fixed rows-per-wave split would idle most
// waves; here each pass spans up to kPairCB column tiles and its (tile row,
// column tile) pairs are dealt to all waves, up to PW per wave.  Both
// fragments of every MFMA come from LDS.
constexpr int kPairCB = 8;

template <typename T, typename M, int NT>
__device__ void wg_same_pairs(const BInst &I, const T *__restrict__ c, T *__restrict__ out, int kp,
                              char *lds, int tr0, int tr1) {
  static_assert(M::KPL == 1 && M::KSTEP == 4, "dense same-spin GEMM uses 16x16x4 MFMA");
  using Frag = typename M::Frag;
  using Out = typename M::Out;
  constexpr int NW = NT / 64;
  constexpr int PW = 8;
  constexpr int TMMAX = (BMAX_NS + 15) / 16;
  const int nsa = I.ns_a, nsb = I.ns_b;
  const int tm = tr1 - tr0, tn = (nsb + 15) / 16;
  const int mp = tm * 16, row0 = tr0 * 16;
  int cbp = (NW * PW) / (tm > 0 ? tm : 1);
  cbp = cbp > kPairCB ? kPairCB : cbp;
  cbp = cbp > tn ? tn : cbp;
  cbp = cbp < 1 ? 1 : cbp;
  const int lda = kp + 1, ldb = cbp * 16 + 1;
  T *Ap = reinterpret_cast<T *>(lds);                 // [mp][lda]
  T *Bp = Ap + (size_t)(TMMAX * 16) * lda;            // [kp][ldb]
  const T *Ha = DenseH<T>::a(I), *Hb = DenseH<T>::b(I);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, li = lane & 15, g = lane >> 4;
  for (int n0 = 0; n0 < tn && tm > 0; n0 += cbp) {
    const int ncb = tn - n0 < cbp ? tn - n0 : cbp;
    const int np = tm * ncb;
    Out acc[PW];
#pragma unroll
    for (int j = 0; j < PW; ++j) acc[j] = Out{0, 0, 0, 0};
    for (int prod = 0; prod < 2; ++prod) {
      const int K = prod == 0 ? nsb : nsa;
      for (int k0 = 0; k0 < K; k0 += kp) {
        for (int e = tid; e < mp * kp; e += NT) {
          const int r = e / kp, k = e - r * kp, kk = k0 + k, rr = row0 + r;
          T v = (T)0;
          if (rr < nsa && kk < K) v = prod == 0 ? c[(int64_t)rr * nsb + kk] : Ha[(int64_t)rr * nsa + kk];
          Ap[r * lda + k] = v;
        }
        for (int e = tid; e < kp * ncb * 16; e += NT) {
          const int k = e / (ncb * 16), j = e - k * (ncb * 16), kk = k0 + k, col = n0 * 16 + j;
          T v = (T)0;
          if (kk < K && col < nsb)
            v = prod == 0 ? Hb[(int64_t)kk * nsb + col] : c[(int64_t)kk * nsb + col];
          Bp[k * ldb + j] = v;
        }
        __syncthreads();
        for (int ks = 0; ks < kp / 4; ++ks) {
#pragma unroll
          for (int j = 0; j < PW; ++j) {
            const int p = wv + NW * j;
            if (p < np) {
              const int tr = p % tm, cv = p / tm;
              const Frag a = Ap[(tr * 16 + li) * lda + ks * 4 + g];
              const Frag b = Bp[(ks * 4 + g) * ldb + cv * 16 + li];
              acc[j] = M::mma(a, b, acc[j]);
            }
          }
        }
        __syncthreads();
      }
    }
#pragma unroll
    for (int j = 0; j < PW; ++j) {
      const int p = wv + NW * j;
      if (p < np) {
        const int tr = p % tm, cv = p / tm;
        const int col = (n0 + cv) * 16 + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = row0 + tr * 16 + M::orow(g, r);
          if (row < nsa && col < nsb) out[(int64_t)row * nsb + col] = (T)acc[j][r];
        }
      }
    }
  }
  __syncthreads();
}

template <typename M>
struct WSel;
template <>
struct WSel<MF64> {
  __device__ static const double *w(const BInst &I) { return I.W64; }
};
template <>
struct WSel<MF32> {
  __device__ static const float *w(const BInst &I) { return I.W32; }
};
template <>
struct WSel<MBF16> {
  __device__ static const __bf16 *w(const BInst &I) { return I.Wbf; }
};

constexpr size_t kWBytes = sizeof(double) * BMAX_NP * BMAX_NP;  // LDS copy of the pair ERI matrix

// out = H c for one vector of instance I (T = double: FP64 everywhere;
// T = float: FP32 same-spin part, MFMA flavour M for the opposite spin).
// Rows [tm.a0, tm.a1) of out = H c for one vector of instance I (c: all
// rows, complete before the call).
template <typename T, typename M, int NT>
__device__ void wg_sigma(const BInst &I, const BParams &P, const T *__restrict__ c,
                         T *__restrict__ out, char *lds, uint64_t *tick, const Team &tm) {
  uint64_t tk = __builtin_amdgcn_s_memrealtime();
  const int tid = threadIdx.x;
  const int nsa = I.ns_a, nsb = I.ns_b;
  // (1) one-electron and same-spin parts of both spins (dense MFMA products)
  if (tm.T > 1) {
    if constexpr (std::is_same<T, double>::value)
      wg_same_pairs<double, MF64, NT>(I, c, out, P.kp, lds, tm.t0, tm.t1);
    else
      wg_same_pairs<float, MF32, NT>(I, c, out, P.kp, lds, tm.t0, tm.t1);
  } else {
    if constexpr (std::is_same<T, double>::value)
      wg_same_dense<double, MF64, NT>(I, c, out, P.kp, lds, 0, (I.ns_a + 15) / 16);
    else
      wg_same_dense<float, MF32, NT>(I, c, out, P.kp, lds, 0, (I.ns_a + 15) / 16);
  }
  if (threadIdx.x == 0) {
    const uint64_t t = __builtin_amdgcn_s_memrealtime();
    tick[0] += t - tk;
    tk = t;
  }
  // (3) opposite spin.  Each wavefront owns the rows Ia = wave, wave + NW, ...:
  // the signed ERI tile of the row's s alpha excitations sits in its
  // registers (A fragments, built from an LDS copy of the pair matrix), the
  // s gathered rows of C stream in as B fragments 16 columns at a time, and
  // every M[kl][J] is scattered through the beta pair table into the wave's
  // own LDS copy of sigma's row.  No workgroup barrier inside the phase.
  using A = typename M::A;
  using Frag = typename M::Frag;
  using Out = typename M::Out;
  constexpr int NW = NT / 64;
  constexpr int KSMAX = (BMAX_S + M::KSTEP - 1) / M::KSTEP;
  constexpr int NPT = BMAX_NP / 16;
  const int np = I.npair;
  A *Wl = reinterpret_cast<A *>(lds);
  double *rows = reinterpret_cast<double *>(lds + kWBytes);
  {
    const A *W = WSel<M>::w(I);
    for (int e = tid; e < np * np; e += NT) Wl[e] = W[e];
  }
  __syncthreads();
  const int lane = tid & 63, wv = tid >> 6, li = lane & 15, g = lane >> 4;
  double *sigw = rows + wv * BMAX_NS;
  const int njt = (nsb + 15) / 16;
  const int sa = I.s_a;
  // The K and pair-tile loops run at the largest shape (the norb = 10
  // instances that bound the makespan use all of it): padded K slots carry
  // zero ERI fragments and padded pair rows carry invalid scatter codes.
  for (int ia = tm.a0 + wv; ia < tm.a1 && sa > 0; ia += NW) {
    const Ent *te = I.tab_a + (int64_t)ia * sa;
    uint32_t boff[KSMAX][M::KPL];
    Frag af[NPT][KSMAX];
#pragma unroll
    for (int ks = 0; ks < KSMAX; ++ks) {
#pragma unroll
      for (int t = 0; t < M::KPL; ++t) {
        const int e = ks * M::KSTEP + g * M::KPL + t;
        const Ent en = te[e < sa ? e : sa - 1];
        const bool ok = e < sa;
        // padded K: the last entry's row (one this row gathers), so that
        // 0 * (a non-finite value) reaches no row that does not gather it
        boff[ks][t] = (uint32_t)en.J * (uint32_t)nsb;
        const int pk = pair_index(en.p, en.q);
        const double sg = !ok ? 0.0 : en.sign < 0 ? -1.0 : 1.0;
#pragma unroll
        for (int u = 0; u < NPT; ++u) {
          const int kl = u * 16 + li;
          const double w = kl < np ? sg * (double)Wl[kl * np + pk] : 0.0;
          if constexpr (M::KPL == 1)
            af[u][ks] = M::cvt(w);
          else
            af[u][ks][t] = M::cvt(w);
        }
      }
    }
    for (int j = lane; j < nsb; j += 64) sigw[j] = 0;
    // column tile jt + 1's B fragments and scatter codes are fetched before
    // tile jt's MFMAs and scatter, so their latency overlaps that work
    // (past the last tile a clamped, valid column is fetched and not used)
    const uint4 *quads = std::is_same<typename M::A, double>::value ? I.quad_s_b : I.quad_r_b;
    const uint32_t qs = (uint32_t)I.ns_pad_b;
    Frag bn[KSMAX];
    uint4 qn[NPT];
    {
      const uint32_t jc = (uint32_t)(li < nsb ? li : nsb - 1);
#pragma unroll
      for (int ks = 0; ks < KSMAX; ++ks) bn[ks] = M::load_b(c, boff[ks], jc);
#pragma unroll
      for (int u = 0; u < NPT; ++u) qn[u] = quads[((uint32_t)u * 4u + (uint32_t)g) * qs + (uint32_t)li];
    }
    for (int jt = 0; jt < njt; ++jt) {
      Frag bf[KSMAX];
      uint4 q[NPT];
#pragma unroll
      for (int ks = 0; ks < KSMAX; ++ks) bf[ks] = bn[ks];
#pragma unroll
      for (int u = 0; u < NPT; ++u) q[u] = qn[u];
      {
        const int jn = (jt + 1) * 16 + li;
        const uint32_t jc = (uint32_t)(jn < nsb ? jn : nsb - 1);
        const uint32_t jq = (uint32_t)(jn < (int)qs ? jn : (int)qs - 1);
#pragma unroll
        for (int ks = 0; ks < KSMAX; ++ks) bn[ks] = M::load_b(c, boff[ks], jc);
#pragma unroll
        for (int u = 0; u < NPT; ++u) qn[u] = quads[((uint32_t)u * 4u + (uint32_t)g) * qs + jq];
      }
#pragma unroll
      for (int u = 0; u < NPT; ++u) {
        Out o = {0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < KSMAX; ++ks) o = M::mma(af[u][ks], bf[ks], o);
        const uint32_t cds[4] = {q[u].x, q[u].y, q[u].z, q[u].w};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const uint32_t code = cds[r];
          if (code != kInvalid) {
            const double val = (double)o[r];
            atomicAdd(&sigw[code >> 1], (code & 1u) ? -val : val);
          }
        }
      }
    }
    for (int j = lane; j < nsb; j += 64) {
      T *o = out + (int64_t)ia * nsb + j;
      *o = (T)((double)*o + sigw[j]);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) tick[1] += __builtin_amdgcn_s_memrealtime() - tk;
}

// ------------------------------------------------------------ vector passes
template <typename T>
struct Vecs {
  T *base;
  int64_t n;
  const int *map;
  __device__ T *operator()(int slot) const { return base + (int64_t)map[slot] * n; }
  __device__ T *xc(int j) const { return base + (int64_t)(NVW + j) * n; }
};

template <typename T>
__device__ const T *diag(const BInst &I);
template <>
__device__ const double *diag<double>(const BInst &I) { return I.D64; }
template <>
__device__ const float *diag<float>(const BInst &I) { return I.D32; }

template <typename T>
__device__ Vecs<T> vecs(const BInst &I, const Ctl &C);
template <>
__device__ Vecs<double> vecs<double>(const BInst &I, const Ctl &C) { return {I.v64, I.ndet, C.m64}; }
template <>
__device__ Vecs<float> vecs<float>(const BInst &I, const Ctl &C) { return {I.v32, I.ndet, C.m32}; }

struct Upd {
  double b, c, E, inv, E0, fl, sx;
  int sy, read_z, nconv, want_zdots;
};

// Fused SBCI update (Eqs. S56-S60 with Eq. S31's preconditioner), the same
// per-element arithmetic as the full-size k_update.  Results in C.h1.
template <typename T, int NT>
__device__ void wg_update(const BInst &I, Ctl &C, Red<NT> &R, const Team &tm, const Upd &a, int zslot,
                          int wslot) {
  const Vecs<T> V = vecs<T>(I, C);
  T *x = V(SX), *X = V(SXX), *y = V(SY), *Y = V(SYY), *w = V(wslot);
  const T *zz = V(zslot);
  const T *Z = V(SZ);
  const T *D = diag<T>(I);
  double v[10 + BMAXR];
#pragma unroll
  for (int q = 0; q < 10 + BMAXR; ++q) v[q] = 0;
  for (int64_t i = tm.r0 + threadIdx.x; i < tm.r1; i += NT) {
    double zi = 0, Zi = 0, yi = 0, Yi = 0;
    if (a.read_z) {
      zi = (double)zz[i];
      Zi = (double)Z[i];
    }
    if (a.sy) {
      yi = (double)y[i];
      Yi = (double)Y[i];
    }
    const double yn = yi - a.c * zi, Yn = Yi - a.c * Zi;
    const double xn = a.sx * (double)x[i] + a.b * yn, Xn = a.sx * (double)X[i] + a.b * Yn;
    const double r = (Xn - a.E * xn) * a.inv;
    double den = (double)D[i] - a.E0;
    if (fabs(den) < a.fl) den = a.fl;
    const double wi = r / den;
    x[i] = (T)xn;
    X[i] = (T)Xn;
    y[i] = (T)yn;
    Y[i] = (T)Yn;
    w[i] = (T)wi;
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
    for (int j = 0; j < BMAXR; ++j)
      if (j < a.nconv) v[10 + j] += ws * (double)V.xc(j)[i];
  }
  wg_sum<NT>(v, 10 + a.nconv, R, tm);
  if ((int)threadIdx.x < 10 + a.nconv) C.h1[threadIdx.x] = R.out[threadIdx.x];
  __syncthreads();
}

// z = w - sum_j d_j xc_j in place (Eq. S31), d_j = C.h1[10 + j]; x.z, y.z, z.z -> C.h2
template <typename T, int NT>
__device__ void wg_deflate(const BInst &I, Ctl &C, Red<NT> &R, const Team &tm, int wslot) {
  const Vecs<T> V = vecs<T>(I, C);
  T *w = V(wslot);
  const T *x = V(SX), *y = V(SY);
  double dj[BMAXR];
#pragma unroll
  for (int j = 0; j < BMAXR; ++j) dj[j] = j < C.nconv ? C.h1[10 + j] : 0.0;
  double v[3] = {0, 0, 0};
  for (int64_t i = tm.r0 + threadIdx.x; i < tm.r1; i += NT) {
    double zi = (double)w[i];
#pragma unroll
    for (int j = 0; j < BMAXR; ++j)
      if (j < C.nconv) zi -= dj[j] * (double)V.xc(j)[i];
    const T zt = (T)zi;
    w[i] = zt;
    const double zs = (double)zt;
    v[0] += (double)x[i] * zs;
    v[1] += (double)y[i] * zs;
    v[2] += zs * zs;
  }
  wg_sum<NT>(v, 3, R, tm);
  if (threadIdx.x < 3) C.h2[threadIdx.x] = R.out[threadIdx.x];
  __syncthreads();
}

// x.Z, y.Z, z.Z -> C.h3
template <typename T, int NT>
__device__ void wg_dots_xyz(const BInst &I, Ctl &C, Red<NT> &R, const Team &tm, int zslot) {
  const Vecs<T> V = vecs<T>(I, C);
  const T *x = V(SX), *y = V(SY), *z = V(zslot), *Z = V(SZ);
  double v[3] = {0, 0, 0};
  for (int64_t i = tm.r0 + threadIdx.x; i < tm.r1; i += NT) {
    const double Zi = (double)Z[i];
    v[0] += (double)x[i] * Zi;
    v[1] += (double)y[i] * Zi;
    v[2] += (double)z[i] * Zi;
  }
  wg_sum<NT>(v, 3, R, tm);
  if (threadIdx.x < 3) C.h3[threadIdx.x] = R.out[threadIdx.x];
  __syncthreads();
}

// Up to BMAXR + 1 vectors with coefficients, passed by value so that the
// unrolled loops below keep them in registers.
template <typename T>
struct Pack {
  const T *p[BMAXR + 1];
  double c[BMAXR + 1];
  int n;
};

// dot products a . b_j over all rows -> R.out[j]
template <typename T, int NT>
__device__ void wg_dots(const Team &tm, const T *a, const Pack<T> bs, Red<NT> &R) {
  double v[BMAXR + 1];
#pragma unroll
  for (int j = 0; j < BMAXR + 1; ++j) v[j] = 0;
  for (int64_t i = tm.r0 + threadIdx.x; i < tm.r1; i += NT) {
    const double ai = (double)a[i];
#pragma unroll
    for (int j = 0; j < BMAXR + 1; ++j)
      if (j < bs.n) v[j] += ai * (double)bs.p[j][i];
  }
  wg_sum<NT>(v, bs.n, R, tm);
}

// out = beta * out + sum_q c_q * x_q (elementwise over this workgroup's rows;
// out may alias one of x_q)
template <typename T, int NT>
__device__ void wg_lincomb(const Team &tm, T *out, const Pack<T> xs, double beta) {
  for (int64_t i = tm.r0 + threadIdx.x; i < tm.r1; i += NT) {
    double s = beta == 0.0 ? 0.0 : beta * (double)out[i];
#pragma unroll
    for (int q = 0; q < BMAXR + 1; ++q)
      if (q < xs.n) s += xs.c[q] * (double)xs.p[q][i];
    out[i] = (T)s;
  }
  __syncthreads();
}

template <typename T>
__device__ Pack<T> pack(int n) {
  Pack<T> k;
#pragma unroll
  for (int j = 0; j < BMAXR + 1; ++j) {
    k.p[j] = nullptr;
    k.c[j] = 0;
  }
  k.n = n;
  return k;
}

template <typename Td, typename Ts, int NT>
__device__ void wg_convert(const Team &tm, Td *dst, const Ts *src, double scale) {
  for (int64_t i = tm.r0 + threadIdx.x; i < tm.r1; i += NT) dst[i] = (Td)(scale * (double)src[i]);
  __syncthreads();
}

// ------------------------------------------------------------ the SBCI1 state machine
template <int NT>
struct Solve {
  const BInst &I;
  const BParams &P;
  Ctl &C;
  Red<NT> &R;
  char *lds;
  Team tm;

  __device__ bool lane0() const { return threadIdx.x == 0; }
  // lane 0 of member 0 writes the instance's outputs
  __device__ bool writer() const { return threadIdx.x == 0 && tm.m == 0; }

  template <typename T>
  __device__ void sigma_phase(const T *c, T *o, int mode) {
    if (tm.T > 1) team_sync<NT>(tm, R);  // every member's rows of c are written
    if constexpr (std::is_same<T, double>::value) {
      wg_sigma<double, MF64, NT>(I, P, c, o, lds, C.tsig, tm);
      if (lane0()) C.nsig64 += 1;
    } else {
      if (mode == SBCI_BF16)
        wg_sigma<float, MBF16, NT>(I, P, c, o, lds, C.tsig, tm);
      else
        wg_sigma<float, MF32, NT>(I, P, c, o, lds, C.tsig, tm);
      if (lane0()) C.nsiglow += 1;
    }
    __syncthreads();
  }

  __device__ double shift(double Enew) const { return C.alpha == 0 ? Enew : C.Ec[0]; }

  template <typename T>
  __device__ void segment_start(double sx) {
    Upd a{};
    a.b = 0;
    a.c = 0;
    a.E = C.E;
    a.inv = 1.0;
    a.E0 = shift(C.E);
    a.fl = P.floor;
    a.sx = sx;
    a.sy = 0;
    a.read_z = 0;
    a.nconv = C.nconv;
    a.want_zdots = C.nconv == 0;
    // the preconditioned residual goes to the current z slot (za)
    wg_update<T, NT>(I, C, R, tm, a, SZB, SZA);
    if (C.nconv > 0) wg_deflate<T, NT>(I, C, R, tm, SZA);
    if (lane0()) {
      C.sx = 1.0;
      C.seg_start = 1;
      C.t = 0;
    }
    __syncthreads();
  }

  // the root start of Algorithm 1 (Eqs. S4-S7); returns false on a vanished vector
  template <typename T>
  __device__ bool start_root() {
    const Vecs<T> V = vecs<T>(I, C);
    T *x = V(SX), *X = V(SXX);
    const int nc = C.nconv;
    if (nc > 0) {
      Pack<T> px = pack<T>(nc), pX = pack<T>(nc);
#pragma unroll
      for (int j = 0; j < BMAXR; ++j) {
        px.p[j] = pX.p[j] = V.xc(j);
      }
      wg_dots<T, NT>(tm, x, px, R);
#pragma unroll
      for (int j = 0; j < BMAXR; ++j) {
        if (j < nc) {
          px.c[j] = -R.out[j];
          pX.c[j] = -C.Ec[j] * R.out[j];
        }
      }
      __syncthreads();
      wg_lincomb<T, NT>(tm, x, px, 1.0);   // Eq. S4
      wg_lincomb<T, NT>(tm, X, pX, 1.0);   // Eq. S5
    }
    Pack<T> p1 = pack<T>(1);
    p1.p[0] = x;
    wg_dots<T, NT>(tm, x, p1, R);
    const double nxx = R.out[0];
    __syncthreads();
    if (!(nxx > 0) || !isfinite(nxx)) return false;
    if (lane0()) {
      C.seg = 0;
      C.steps_root = 0;
      C.stall = 0;
      C.bestE = C.E;
    }
    __syncthreads();
    segment_start<T>(1.0 / sqrt(nxx));  // Eqs. S6-S7, applied lazily
    return true;
  }

  // E = x.X / x.x of the current vectors of precision T
  template <typename T>
  __device__ double rayleigh() {
    const Vecs<T> V = vecs<T>(I, C);
    Pack<T> bs = pack<T>(2);
    bs.p[0] = V(SX);
    bs.p[1] = V(SXX);
    wg_dots<T, NT>(tm, V(SX), bs, R);
    const double e = R.out[1] / R.out[0];
    __syncthreads();
    return e;
  }

  __device__ bool to_f32() {
    const Vecs<float> V = vecs<float>(I, C);
    sigma_phase<float>(V(SX), V(SXX), SBCI_F32);
    const double e = rayleigh<float>();
    const int steps = C.steps_root, seg = C.seg;
    if (lane0()) {
      C.E = e;
      C.phase = SBCI_F32;
    }
    __syncthreads();
    if (!start_root<float>()) return false;
    if (lane0()) {
      C.steps_root = steps;
      C.seg = seg + 1;
    }
    __syncthreads();
    return true;
  }

  __device__ bool promote() {
    const Vecs<double> V = vecs<double>(I, C);
    const Vecs<float> F = vecs<float>(I, C);
    wg_convert<double, float, NT>(tm, V(SX), F(SX), 1.0);
    sigma_phase<double>(V(SX), V(SXX), SBCI_F64);
    const double e = rayleigh<double>();
    const int steps = C.steps_root, seg = C.seg;
    if (lane0()) {
      C.E = e;
      C.phase = SBCI_F64;
    }
    __syncthreads();
    if (!start_root<double>()) return false;
    if (lane0()) {
      C.steps_root = steps;
      C.seg = seg + 1;
    }
    __syncthreads();
    return true;
  }

  // Converged root (FP64): store x_c, then the next root's start from the
  // second Ritz vector of this step (Section S1.4).  Returns false on error.
  __device__ bool finish_root(double xn, bool second_ok) {
    const Vecs<double> V = vecs<double>(I, C);
    const int j = C.nconv;
    wg_convert<double, double, NT>(tm, V.xc(j), V(SX), 1.0 / xn);
    if (P.precision != SBCI_F64) {
      const Vecs<float> F = vecs<float>(I, C);
      wg_convert<float, double, NT>(tm, F.xc(j), V.xc(j), 1.0);
    }
    if (lane0()) {
      C.Ec[j] = C.E;
      C.nconv = j + 1;
      if (C.nconv >= I.nroots) C.done = 1;
    }
    __syncthreads();
    if (C.done) return true;
    if (!second_ok) {
      if (lane0()) C.status = SBCI_ENUMERIC;
      __syncthreads();
      return false;
    }
    const double ax = C.last.a2[0], ay = C.last.a2[1], az = C.last.a2[2];
    const double b = C.last.b, c = C.last.c;
    Pack<double> in1 = pack<double>(3), in2 = pack<double>(3);
    in1.c[0] = in2.c[0] = ax;
    in1.c[1] = in2.c[1] = ay - ax * b;
    in1.c[2] = in2.c[2] = ay * c + az;
    in1.p[0] = V(SX);
    in1.p[1] = V(SY);
    in1.p[2] = V(SZA);
    in2.p[0] = V(SXX);
    in2.p[1] = V(SYY);
    in2.p[2] = V(SZ);
    wg_lincomb<double, NT>(tm, V(SZB), in1, 0.0);
    wg_lincomb<double, NT>(tm, V(SYY), in2, 0.0);
    if (lane0()) {
      int t = C.m64[SX];
      C.m64[SX] = C.m64[SZB];
      C.m64[SZB] = t;
      t = C.m64[SXX];
      C.m64[SXX] = C.m64[SYY];
      C.m64[SYY] = t;
      C.E = C.last.E[1];
      C.alpha += 1;
    }
    __syncthreads();
    if (P.precision != SBCI_F64) {
      const Vecs<double> V2 = vecs<double>(I, C);
      const Vecs<float> F = vecs<float>(I, C);
      wg_convert<float, double, NT>(tm, F(SX), V2(SX), 1.0);
      wg_convert<float, double, NT>(tm, F(SXX), V2(SXX), 1.0);
      if (lane0()) C.phase = P.precision;
      __syncthreads();
      return start_root<float>();
    }
    if (lane0()) C.phase = SBCI_F64;
    __syncthreads();
    return start_root<double>();
  }

  template <typename T>
  __device__ bool restart_from_ritz() {
    const RitzS r = C.r;
    const Vecs<T> V = vecs<T>(I, C);
    Pack<T> in1 = pack<T>(3), in2 = pack<T>(3);
    in1.c[0] = in2.c[0] = r.a1[0] * C.sx;
    in1.c[1] = in2.c[1] = C.seg_start ? 0.0 : r.a1[1];
    in1.c[2] = in2.c[2] = r.a1[2];
    in1.p[0] = V(SX);
    in1.p[1] = V(SY);
    in1.p[2] = V(SZA);
    in2.p[0] = V(SXX);
    in2.p[1] = V(SYY);
    in2.p[2] = V(SZ);
    // the Ritz vector goes to the free z slot; x and X stay intact until its
    // norm is known to be usable
    wg_lincomb<T, NT>(tm, V(SZB), in1, 0.0);
    Pack<T> pv = pack<T>(1);
    pv.p[0] = V(SZB);
    wg_dots<T, NT>(tm, V(SZB), pv, R);
    const double nxx = R.out[0];
    __syncthreads();
    if (!(nxx > 0) || !isfinite(nxx)) {
      if (C.phase == SBCI_BF16) return to_f32();
      if (C.phase != SBCI_F64) return promote();
      if (lane0()) C.status = SBCI_ENUMERIC;
      __syncthreads();
      return false;
    }
    wg_lincomb<T, NT>(tm, V(SYY), in2, 0.0);
    if (lane0()) {
      int *m = std::is_same<T, double>::value ? C.m64 : C.m32;
      int t = m[SX];
      m[SX] = m[SZB];
      m[SZB] = t;
      t = m[SXX];
      m[SXX] = m[SYY];
      m[SYY] = t;
      C.E = r.E[0];
      C.seg += 1;
      C.nrestarts += 1;
    }
    __syncthreads();
    segment_start<T>(1.0 / sqrt(nxx));
    return true;
  }

  // One SBCI step of the running root in precision T.  Returns false when
  // the instance stops with an error (C.status set).
  template <typename T>
  __device__ bool step() {
    const Vecs<T> V = vecs<T>(I, C);
    const int mode = C.phase;
    sigma_phase<T>(V(SZA), V(SZ), mode);                       // Eq. S32
    wg_dots_xyz<T, NT>(I, C, R, tm, SZA);
    if (lane0()) {
      C.steps_root += 1;
      C.nsteps += 1;
      const double sx = C.sx;
      double N[6], Hm[6];
      N[0] = sx * sx * C.h1[1];
      N[1] = sx * C.h1[2];
      N[3] = C.h1[3];
      Hm[0] = sx * sx * C.h1[4];
      Hm[1] = sx * C.h1[5];
      Hm[3] = C.h1[6];
      if (C.nconv > 0) {
        N[2] = sx * C.h2[0];
        N[4] = C.h2[1];
        N[5] = C.h2[2];
      } else {
        N[2] = sx * C.h1[7];
        N[4] = C.h1[8];
        N[5] = C.h1[9];
      }
      Hm[2] = sx * C.h3[0];
      Hm[4] = C.h3[1];
      Hm[5] = C.h3[2];
      bool fin = true;
      for (int i = 0; i < 6; ++i) fin = fin && isfinite(N[i]) && isfinite(Hm[i]);
      // action: 0 update, 1 error, 2 finish (eigenvector at segment start),
      // 3 promote, 4 new segment (rank), 5 restart from Ritz, 6 hand over to
      // the next precision rung
      if (!fin) {
        // a low-precision phase hands over (X = H x is recomputed from x)
        if (C.phase != SBCI_F64) {
          C.action = 6;
        } else {
          C.action = 1;
          C.status = SBCI_ENUMERIC;
        }
      } else {
        C.r = pod(C.seg_start ? ritz_first(N[0], N[2], N[5], Hm[0], Hm[2], Hm[5], P.lindep)
                              : ritz_next(N, Hm, P.lindep));
        if (!C.r.rank_ok) {
          if (C.seg_start) {
            const double dz0 = sqrt(C.h1[0]);
            if (C.phase == SBCI_F64 && dz0 < P.r0) {
              C.action = 2;
              C.dzroot = dz0;
            } else if (C.phase != SBCI_F64) {
              C.action = 3;
            } else {
              C.action = 1;
              C.status = SBCI_ENUMERIC;
            }
          } else if (!(N[0] > 0)) {
            if (C.phase != SBCI_F64) {
              C.action = 6;
            } else {
              C.action = 1;
              C.status = SBCI_ENUMERIC;
            }
          } else {
            C.action = 4;
            C.nrestarts += 1;
            C.seg += 1;
            C.dzroot = sx / sqrt(N[0]);
          }
        } else if (!C.r.coef_ok) {
          C.action = 5;
        } else if (C.phase != SBCI_F64 && fabs(C.r.k) < P.x_th1) {
          // |x_{t+1}| = |k_t|: the update would build x_{t+1} by heavy
          // cancellation, which the low-precision images cannot follow; the
          // phase hands over from the current, intact x
          C.action = 6;
        } else {
          C.action = 0;
        }
      }
    }
    __syncthreads();
    const int act = C.action;
    if (act == 1) return false;
    if (act == 2) {
      if (lane0()) C.h2[3] = C.dzroot;  // residual of the finished root
      __syncthreads();
      return finish_root(sqrt(C.h1[1]), false);
    }
    if (act == 3) return promote();
    if (act == 4) {
      segment_start<T>(C.dzroot);
      return true;
    }
    if (act == 5) return restart_from_ritz<T>();
    if (act == 6) return C.phase == SBCI_BF16 ? to_f32() : promote();
    const RitzS r = C.r;
    const double Enew = r.E[0];
    Upd a{};
    a.b = r.b;
    a.c = r.c;
    a.E = Enew;
    a.inv = 1.0 / fabs(r.k);
    a.E0 = shift(Enew);
    a.fl = P.floor;
    a.sx = C.sx;
    a.sy = C.seg_start ? 0 : 1;
    a.read_z = 1;
    a.nconv = C.nconv;
    a.want_zdots = C.nconv == 0;
    wg_update<T, NT>(I, C, R, tm, a, SZA, SZB);
    // decisions (lane 0), then the follow-up passes
    if (lane0()) {
      C.last = r;
      const double dz = sqrt(C.h1[0]);
      const double xn = sqrt(C.h1[1]);
      const double dE = fabs(Enew - C.E);
      C.dzroot = dz;
      C.h2[3] = xn;
      int act2 = 0;  // 0 continue, 1 error, 2 converged, 3 hand-over, 4 cap
      if (!isfinite(dz) || !isfinite(xn) || !isfinite(Enew)) {
        act2 = 1;
        C.status = SBCI_ENUMERIC;
      } else {
        int reason = 0;
        bool conv = false, prom = false;
        const bool low = C.phase != SBCI_F64;
        if (!low && dE < P.eps0 && dz < P.r0) {
          conv = true;
          reason = 1;
        } else if (low) {
          if (Enew < C.bestE - 1e-15 * fabs(C.bestE)) {
            C.bestE = Enew;
            C.stall = 0;
          } else {
            C.stall += 1;
          }
          const bool bf = C.phase == SBCI_BF16;
          const double e0 = bf ? P.bf16_eps0 : P.mix_eps0, r0 = bf ? P.bf16_r0 : P.mix_r0;
          if ((dE < e0 && dz < r0) || C.stall >= P.mix_stall) {
            prom = true;
            reason = 8;
          }
        }
        if (!conv && !prom) {
          const bool s62a = C.alpha > 0 && fabs(r.b) < P.b_th && dE < P.eps1;
          const bool s62b = xn < P.x_th1 || xn > P.x_th2;
          const bool s62c = dz > P.r1 && C.t > 0;
          const bool cap = C.t + 1 >= P.max_cycle;
          reason = s62a ? 2 : s62b ? 3 : s62c ? 4 : cap ? 5 : 0;
        }
        C.E = Enew;
        if (conv) {
          act2 = 2;
        } else if (prom) {
          act2 = 3;
        } else if (C.steps_root >= P.max_steps) {
          C.any_noconv = 1;
          act2 = 4;
        } else {
          if (reason >= 2) {
            C.nrestarts += 1;
            C.seg += 1;
            C.t = 0;
            C.seg_start = 1;
            C.sx = 1.0 / xn;
          } else {
            C.t += 1;
            C.seg_start = 0;
            C.sx = 1.0;
          }
        }
      }
      C.action = act2;
    }
    __syncthreads();
    const int act2 = C.action;
    const double xn = C.h2[3];
    if (act2 == 1) return false;
    if (act2 == 2) return finish_root(xn, true);
    if (act2 == 3) return C.phase == SBCI_BF16 ? to_f32() : promote();
    if (act2 == 4) {
      if (C.phase != SBCI_F64) return promote();
      return finish_root(xn, true);
    }
    if (C.nconv > 0) wg_deflate<T, NT>(I, C, R, tm, SZB);
    if (lane0()) {
      int *m = std::is_same<T, double>::value ? C.m64 : C.m32;
      const int t = m[SZA];
      m[SZA] = m[SZB];
      m[SZB] = t;
    }
    __syncthreads();
    return true;
  }

  // Section S1.1: the k lowest diagonal determinants (ties: lower index),
  // sigma on their unit vectors, k x k eigenproblem; x, X from its lowest
  // eigenvector.  He_i are kept in the y, Y, za, zb slots (k <= 4).  Every
  // team member scans the whole diagonal (the same picks everywhere); the
  // entries (He_q)[idx_i] come from their owners through a team sum.
  __device__ bool initial_vector() {
    const Vecs<double> V = vecs<double>(I, C);
    const int k = (int)(I.nroots < I.ndet ? I.nroots : I.ndet);
    const double *D = I.D64;
    for (int q = 0; q < k; ++q) {
      double bv = INFINITY;
      int64_t bi = INT64_MAX;
      for (int64_t i = threadIdx.x; i < I.ndet; i += NT) {
        bool taken = false;
        for (int p = 0; p < q; ++p) taken = taken || C.idx[p] == i;
        const double d = D[i];
        if (!taken && (d < bv || (d == bv && i < bi))) {
          bv = d;
          bi = i;
        }
      }
      // argmin over the workgroup: (value, index) lexicographic
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(bv, o, 64);
        const int64_t oi = __shfl_xor(bi, o, 64);
        if (ov < bv || (ov == bv && oi < bi)) {
          bv = ov;
          bi = oi;
        }
      }
      if ((threadIdx.x & 63) == 0) {
        R.w[threadIdx.x >> 6][0] = bv;
        R.w[threadIdx.x >> 6][1] = __longlong_as_double(bi);
      }
      __syncthreads();
      if (lane0()) {
        double v0 = R.w[0][0];
        int64_t i0 = __double_as_longlong(R.w[0][1]);
        for (int w = 1; w < NT / 64; ++w) {
          const double v1 = R.w[w][0];
          const int64_t i1 = __double_as_longlong(R.w[w][1]);
          if (v1 < v0 || (v1 == v0 && i1 < i0)) {
            v0 = v1;
            i0 = i1;
          }
        }
        C.idx[q] = i0;
      }
      __syncthreads();
    }
    const int hs[4] = {SY, SYY, SZA, SZB};
    double *x = V(SX);
    for (int q = 0; q < k; ++q) {
      for (int64_t i = tm.r0 + threadIdx.x; i < tm.r1; i += NT) x[i] = i == C.idx[q] ? 1.0 : 0.0;
      __syncthreads();
      sigma_phase<double>(x, V(hs[q]), SBCI_F64);              // Eq. S1
      double hv[BMAXR];
#pragma unroll
      for (int i = 0; i < BMAXR; ++i) {
        const int64_t r = i < k ? C.idx[i] : -1;
        hv[i] = (threadIdx.x == 0 && r >= tm.r0 && r < tm.r1) ? V(hs[q])[r] : 0.0;
      }
      wg_sum<NT>(hv, k, R, tm);
      if ((int)threadIdx.x < k) C.Hs[threadIdx.x * k + q] = R.out[threadIdx.x];
      __syncthreads();
    }
    if (lane0()) {
      for (int i = 0; i < k; ++i)
        for (int j = 0; j < i; ++j)
          C.Hs[i * k + j] = C.Hs[j * k + i] = 0.5 * (C.Hs[i * k + j] + C.Hs[j * k + i]);
      jacobi_eigh<BMAXR>(k, C.Hs, C.w, C.U);
      C.E = C.w[0];
    }
    __syncthreads();
    // x = sum_i U[i][0] e_idx_i (Eq. S2), X = sum_i U[i][0] He_i (Eq. S3)
    for (int64_t i = tm.r0 + threadIdx.x; i < tm.r1; i += NT) {
      double s = 0;
      for (int q = 0; q < k; ++q)
        if (C.idx[q] == i) s += C.U[q * k + 0];
      x[i] = s;
    }
    Pack<double> hp = pack<double>(k);
#pragma unroll
    for (int q = 0; q < BMAXR; ++q) {
      hp.p[q] = V(hs[q]);
      hp.c[q] = q < k ? C.U[q * k + 0] : 0.0;
    }
    wg_lincomb<double, NT>(tm, V(SXX), hp, 0.0);
    return true;
  }

  __device__ void run(BOut &out) {
    if (lane0()) {
      R.gen = 0u;
      R.red = 0u;
      R.abort = 0;
      C.alpha = 0;
      C.seg = 0;
      C.t = 0;
      C.steps_root = 0;
      C.phase = SBCI_F64;
      C.seg_start = 1;
      C.stall = 0;
      C.done = 0;
      C.any_noconv = 0;
      C.nconv = 0;
      C.status = SBCI_OK;
      for (int i = 0; i < NVW; ++i) C.m64[i] = C.m32[i] = i;
      C.nsteps = C.nrestarts = C.nsig64 = C.nsiglow = 0;
      C.tsig[0] = C.tsig[1] = 0;
      C.E = 0;
      C.sx = 1;
      C.bestE = 0;
      for (int i = 0; i < BMAXR; ++i) {
        C.Ec[i] = NAN;
        C.idx[i] = -1;
      }
      C.last = pod(Ritz());
      C.r = pod(Ritz());
    }
    __syncthreads();
    bool ok = initial_vector();
    if (ok) {
      if (P.precision != SBCI_F64) {
        const Vecs<double> V = vecs<double>(I, C);
        const Vecs<float> F = vecs<float>(I, C);
        wg_convert<float, double, NT>(tm, F(SX), V(SX), 1.0);
        wg_convert<float, double, NT>(tm, F(SXX), V(SXX), 1.0);
        if (lane0()) C.phase = P.precision;
        __syncthreads();
        ok = start_root<float>();
      } else {
        ok = start_root<double>();
      }
      if (!ok && lane0()) C.status = SBCI_ENUMERIC;
      __syncthreads();
    }
    // hard bound on the number of passes (every pass is a step or a phase change)
    const int cap = I.nroots * (P.max_steps + 8) + 8;
    int guard = 0;
    int last_nconv = 0;
    while (ok && !C.done && !R.abort && guard < cap) {
      ++guard;
      ok = C.phase == SBCI_F64 ? step<double>() : step<float>();
      if (writer() && C.nconv > last_nconv) out.dz[C.nconv - 1] = C.dzroot;
      last_nconv = C.nconv;
      __syncthreads();
    }
    if (writer()) {
      for (int i = 0; i < BMAXR; ++i) out.E[i] = C.Ec[i];
      out.nconv = C.nconv;
      out.nsteps = C.nsteps;
      out.nrestarts = C.nrestarts;
      out.nsig64 = C.nsig64;
      out.nsiglow = C.nsiglow;
      for (int q = 0; q < 2; ++q) out.tsig[q] = C.tsig[q];
      int st = C.status;
      if (R.abort) st = SBCI_EDEVICE;  // a team member stopped arriving
      else if (st == SBCI_OK && (!C.done || C.any_noconv)) st = SBCI_ENOCONV;
      out.status = st;
    }
    __syncthreads();
  }
};

// Blocks [0, ntw) are team members: team_blk[b] = (instance, T, member,
// team).  They run their team's instance first (they are dispatched first,
// and ntw never exceeds the resident capacity, so every member of a team is
// resident at once), then join the queue.  The queue holds the other
// instances (order[0 .. nqueue)), each run by one workgroup.
template <int NT>
__global__ __launch_bounds__(NT) void k_batch(const BInst *__restrict__ inst,
                                              const int *__restrict__ order, int nqueue,
                                              unsigned *queue, BOut *out,
                                              const BParams *__restrict__ prm,
                                              const int4 *__restrict__ team_blk, int ntw,
                                              TeamSync *tsync) {
  extern __shared__ __align__(16) char lds[];
  __shared__ Ctl C;
  __shared__ Red<NT> R;
  __shared__ int item;
  if ((int)blockIdx.x < ntw) {
    const int4 tb = team_blk[blockIdx.x];
    const BInst &I = inst[tb.x];
    Solve<NT> S{I, *prm, C, R, lds, make_team(I.ns_a, I.ns_b, tsync + tb.w, tb.y, tb.z, prm->team_wait)};
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    S.run(out[tb.x]);
    if (threadIdx.x == 0 && tb.z == 0) {
      out[tb.x].t0 = t0;
      out[tb.x].t1 = __builtin_amdgcn_s_memrealtime();
    }
    __syncthreads();
  }
  for (;;) {
    if (threadIdx.x == 0) item = (int)atomicAdd(queue, 1u);
    __syncthreads();
    const int it = item;
    __syncthreads();
    if (it >= nqueue) break;
    const int id = order[it];
    // descriptors and parameters stay in global memory (uniform loads)
    const BInst &I = inst[id];
    Solve<NT> S{I, *prm, C, R, lds, make_team(I.ns_a, I.ns_b, nullptr, 1, 0, 0)};
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    S.run(out[id]);
    if (threadIdx.x == 0) {
      out[id].t0 = t0;
      out[id].t1 = __builtin_amdgcn_s_memrealtime();
    }
  }
}

// Graph-safe reset of the work queue and of the team barriers (a kernel, not
// a memset node).
__global__ void k_batch_reset(unsigned *queue, TeamSync *tsync, int nteam) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) queue[0] = 0u;
  if (t < nteam) {
    tsync[t].cnt = 0u;
    tsync[t].abort = 0u;
  }
}

// Dense same-spin operator from its lists: H[i][col(i,f)] = F[i][f]
// (H zero-initialised; the list columns of a row are distinct).
__global__ void k_dense(const int32_t *__restrict__ fcol, const double *__restrict__ f64,
                        int64_t ns, int nf, double *__restrict__ d64, float *__restrict__ d32) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= ns * nf) return;
  const int64_t i = e / nf;
  const int64_t j = fcol[e];
  d64[i * ns + j] = f64[e];
  d32[i * ns + j] = (float)f64[e];
}

size_t lds_bytes(int kp, int threads) {
  const int nw = threads / 64;
  const int rw = ((BMAX_NS + 15) / 16 + nw - 1) / nw;
  const int cb = rw >= 8 ? 1 : 8 / rw;
  const size_t same = sizeof(double) * ((size_t)((BMAX_NS + 15) / 16 * 16) * (kp + 1) +
                                        (size_t)kp * (std::max(cb, kPairCB) * 16 + 1));
  const size_t opp = kWBytes + sizeof(double) * BMAX_NS * (size_t)nw;
  return std::max(same, opp);
}

}  // namespace
}  // namespace sbci

// ------------------------------------------------------------ host side
using namespace sbci;

struct SpinT {
  double *d64 = nullptr;  // dense same-spin operator [ns][ns]
  float *d32 = nullptr;
};

struct sbci_batch {
  int ninst = 0;
  int device = 0;
  int ncu = 0;
  hipStream_t stream = nullptr;
  std::vector<sbci_ctx *> ctx;
  std::vector<SpinT> la, lb;  // dense same-spin operators per instance
  std::vector<int> nroots;    // of the last solve
  BInst *d_inst = nullptr;
  BParams *d_params = nullptr;
  int *d_order = nullptr;
  unsigned *d_queue = nullptr;
  int4 *d_team_blk = nullptr;   // [ninst * BMAX_TEAM]
  TeamSync *d_tsync = nullptr;  // [ninst]
  BOut *d_out = nullptr;
  double *arena64 = nullptr;
  float *arena32 = nullptr;
  size_t cap64 = 0, cap32 = 0;
  std::vector<BInst> h_inst;
  sbci_batch_config tuned{};
  bool have_tuned = false;
  int solved_precision = -1;
};

namespace {

int batch_error(int code, const std::string &m) { return set_error(code, m); }

constexpr double kRealtimeHz = 100e6;  // s_memrealtime counter frequency

int build_dense(sbci_batch *b, int i) {
  sbci_ctx *c = b->ctx[i];
  auto mk = [&](const SpinTables &T, SpinT &o) -> int {
    const int64_t n2 = T.ns * T.ns, n = T.ns * T.nf;
    SBCI_HIP(hipMalloc(&o.d64, sizeof(double) * n2));
    SBCI_HIP(hipMalloc(&o.d32, sizeof(float) * n2));
    SBCI_HIP(hipMemsetAsync(o.d64, 0, sizeof(double) * n2, b->stream));
    SBCI_HIP(hipMemsetAsync(o.d32, 0, sizeof(float) * n2, b->stream));
    k_dense<<<(unsigned)((n + 255) / 256), 256, 0, b->stream>>>(T.fcol, T.fval64, T.ns, T.nf, o.d64, o.d32);
    SBCI_CHECK_LAUNCH();
    return SBCI_OK;
  };
  SBCI_TRY(mk(c->A, b->la[i]));
  if (c->B.shared) {
    b->lb[i] = b->la[i];
  } else {
    SBCI_TRY(mk(c->B, b->lb[i]));
  }
  return SBCI_OK;
}

// Workgroups of k_batch<NT> resident at once on the device.
template <int NT>
int resident_blocks(sbci_batch *b, size_t lds, int *out) {
  SBCI_HIP(hipFuncSetAttribute((const void *)k_batch<NT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
  int per_cu = 0;
  SBCI_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_batch<NT>, NT, lds));
  *out = per_cu * b->ncu;
  return SBCI_OK;
}

struct Plan {
  int ntw = 0;     // team workgroups (the first blocks)
  int nteam = 0;
  int nqueue = 0;  // instances in the queue
  int grid = 1;
};

template <int NT>
int instantiate(sbci_batch *b, const Plan &pl, size_t lds, hipGraphExec_t *exec_out,
                hipGraph_t *graph_out) {
  SBCI_HIP(hipFuncSetAttribute((const void *)k_batch<NT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
  const unsigned grid = (unsigned)pl.grid;
  hipGraph_t g = nullptr;
  SBCI_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  k_batch_reset<<<(unsigned)((pl.nteam + 255) / 256 + 1), 256, 0, b->stream>>>(b->d_queue, b->d_tsync,
                                                                              pl.nteam);
  k_batch<NT><<<grid, NT, lds, b->stream>>>(b->d_inst, b->d_order, pl.nqueue, b->d_queue, b->d_out,
                                            b->d_params, b->d_team_blk, pl.ntw, b->d_tsync);
  hipError_t le = hipGetLastError();
  hipError_t e = hipStreamEndCapture(b->stream, &g);
  if (le != hipSuccess) return batch_error(SBCI_EDEVICE, std::string("batch launch: ") + hipGetErrorString(le));
  if (e != hipSuccess) return batch_error(SBCI_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    hipGraphDestroy(g);
    return batch_error(SBCI_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
  }
  *exec_out = x;
  *graph_out = g;
  return SBCI_OK;
}

int check_config(const sbci_batch_config &c) {
  if (c.threads != 256 && c.threads != 512 && c.threads != 1024)
    return batch_error(SBCI_EINVAL, "batch config: threads must be 256, 512 or 1024");
  if (c.wg_per_cu < 1 || c.wg_per_cu > 4)
    return batch_error(SBCI_EINVAL, "batch config: wg_per_cu must be in 1..4");
  if (c.order != 0 && c.order != 1) return batch_error(SBCI_EINVAL, "batch config: order must be 0 or 1");
  if (c.k_panel != 8 && c.k_panel != 16)
    return batch_error(SBCI_EINVAL, "batch config: k_panel must be 8 or 16");
  if (c.max_team < 0 || c.max_team > BMAX_TEAM)
    return batch_error(SBCI_EINVAL, "batch config: max_team must be in 0..4");
  if (c.team_wait_us < 0) return batch_error(SBCI_EINVAL, "batch config: team_wait_us must be >= 0");
  if (c.queue_reserve != 0 && (c.queue_reserve < 2 || c.queue_reserve > 64))
    return batch_error(SBCI_EINVAL, "batch config: queue_reserve must be 0 or in 2..64");
  return SBCI_OK;
}

int params_from(const sbci_opts *opt, double tol, BParams &P, int &precision) {
  sbci_opts o;
  if (opt) o = *opt; else sbci_default_opts(&o);
  if (tol > 0) {
    o.eps0 = tol;
    o.r0 = std::sqrt(tol);
  }
  if (!(o.eps0 > 0) || !(o.r0 > 0)) return batch_error(SBCI_EINVAL, "eps0 and r0 must be > 0");
  if (o.precision != SBCI_F64 && o.precision != SBCI_F32 && o.precision != SBCI_BF16)
    return batch_error(SBCI_EINVAL, "unknown precision");
  if (o.max_cycle < 1 || o.max_steps < 1) return batch_error(SBCI_EINVAL, "max_cycle, max_steps >= 1");
  if (o.x0) return batch_error(SBCI_EINVAL, "batch solve: opts.x0 must be NULL");
  if (o.nconv0 != 0) return batch_error(SBCI_EINVAL, "batch solve: opts.nconv0 must be 0");
  P.eps0 = o.eps0;
  P.r0 = o.r0;
  P.b_th = o.b_th;
  P.eps1 = o.eps1;
  P.x_th1 = o.x_th1;
  P.x_th2 = o.x_th2;
  P.r1 = o.r1;
  P.mix_eps0 = o.mix_eps0;
  P.mix_r0 = o.mix_r0;
  P.bf16_eps0 = o.bf16_eps0;
  P.bf16_r0 = o.bf16_r0;
  P.floor = o.precond_floor;
  P.lindep = o.lindep;
  P.max_cycle = o.max_cycle;
  P.max_steps = o.max_steps;
  P.precision = o.precision;
  P.mix_stall = o.mix_stall;
  precision = o.precision;
  return SBCI_OK;
}

// Per-instance vectors and descriptors for this nroots / precision.
int prepare(sbci_batch *b, const int *nroots, int precision) {
  size_t need64 = 0, need32 = 0;
  for (int i = 0; i < b->ninst; ++i) {
    if (nroots[i] < 1 || nroots[i] > BMAXR || nroots[i] > b->ctx[i]->ndet)
      return batch_error(SBCI_EINVAL, "batch nroots must be in [1, min(4, N_det)] for every instance");
    const size_t n = (size_t)b->ctx[i]->ndet * (size_t)(NVW + nroots[i]);
    need64 += (n + 63) / 64 * 64;
    if (precision != SBCI_F64) need32 += (n + 63) / 64 * 64;
  }
  if (need64 > b->cap64) {
    hipFree(b->arena64);
    b->arena64 = nullptr;
    SBCI_HIP(hipMalloc(&b->arena64, sizeof(double) * need64));
    b->cap64 = need64;
  }
  if (need32 > b->cap32) {
    hipFree(b->arena32);
    b->arena32 = nullptr;
    SBCI_HIP(hipMalloc(&b->arena32, sizeof(float) * need32));
    b->cap32 = need32;
  }
  b->h_inst.resize(b->ninst);
  size_t o64 = 0, o32 = 0;
  for (int i = 0; i < b->ninst; ++i) {
    sbci_ctx *c = b->ctx[i];
    BInst &I = b->h_inst[i];
    I.ns_a = (int)c->A.ns;
    I.ns_b = (int)c->B.ns;
    I.s_a = c->A.s;
    I.s_b = c->B.s;
    I.nf_a = c->A.nf;
    I.nf_b = c->B.nf;
    I.npair = c->npair;
    I.nroots = nroots[i];
    I.ndet = c->ndet;
    I.ns_pad_b = c->B.ns_pad;
    I.tab_a = c->A.tab;
    I.pair_b = c->B.pair;
    I.quad_r_b = c->B.quad_r;
    I.quad_s_b = c->B.quad_s;
    I.H64_a = b->la[i].d64;
    I.H64_b = b->lb[i].d64;
    I.H32_a = b->la[i].d32;
    I.H32_b = b->lb[i].d32;
    I.W64 = c->W64;
    I.W32 = c->W32;
    I.Wbf = reinterpret_cast<const __bf16 *>(c->Wbf);
    I.D64 = c->hdiag;
    I.D32 = c->hdiag32;
    const size_t n = (size_t)c->ndet * (size_t)(NVW + nroots[i]);
    I.v64 = b->arena64 + o64;
    o64 += (n + 63) / 64 * 64;
    if (precision != SBCI_F64) {
      I.v32 = b->arena32 + o32;
      o32 += (n + 63) / 64 * 64;
    } else {
      I.v32 = nullptr;
    }
  }
  SBCI_HIP(hipMemcpyAsync(b->d_inst, b->h_inst.data(), sizeof(BInst) * b->ninst,
                          hipMemcpyHostToDevice, b->stream));
  b->nroots.assign(nroots, nroots + b->ninst);
  return SBCI_OK;
}

constexpr double kTeamMargin = 1.25;
// The teams take at most slots - slots / queue_reserve of the resident
// workgroup slots (16 by default); the rest start on the queue at once (the
// team members join it after their instance).  Fewer reserved slots let
// the teams grow; more let the queue of small instances finish sooner.
// Which bounds the makespan depends on the form (measured on the
// 512-instance workload: FP64 gains from 16, the FP32 ladder from 8), so
// the autotuner tries both.
constexpr int kQueueReserve = 16;

// Estimated work of an instance: N_det x (F lists + opposite-spin pair rows) x roots.
double inst_work(const BInst &I) {
  return (double)I.ndet * (double)(I.nf_a + I.nf_b + I.npair * I.s_a / 2 + 24) * I.nroots;
}

// Launch plan: team sizes, the team block table and the queue order.
// Balanced share M = max(total work / workgroup slots, largest work /
// max_team); an instance of work w gets T = ceil(w / M) workgroups (at most
// max_team), largest first, while the team workgroups fit in the slots that
// are resident at once; slots the rounding leaves unused go to the teams
// with the most work per member.  The other instances form the queue,
// largest first (order 0) or in input order (order 1).
int plan_launch(sbci_batch *b, const sbci_batch_config &cfg, int resident, Plan &pl) {
  const int n = b->ninst;
  const int slots = std::max(1, std::min(b->ncu * cfg.wg_per_cu, resident));
  const int maxT = cfg.max_team == 0 ? BMAX_TEAM : cfg.max_team;
  std::vector<int> ord(n);
  for (int i = 0; i < n; ++i) ord[i] = i;
  std::vector<double> w(n);
  double total = 0, wmax = 0;
  for (int i = 0; i < n; ++i) {
    w[i] = inst_work(b->h_inst[i]);
    total += w[i];
    wmax = std::max(wmax, w[i]);
  }
  std::vector<int> by_work = ord;
  std::stable_sort(by_work.begin(), by_work.end(), [&](int x, int y) { return w[x] > w[y]; });
  std::vector<char> in_team(n, 0);
  std::vector<int4> blk;
  if (maxT > 1 && n > 1) {
    // T_i = ceil(kTeamMargin w_i / M), at most max_team and the instance's
    // alpha tiles (a member needs one); M grows from the balanced share until
    // the teams leave 1/kQueueReserve of the slots to the queue.  The margin
    // covers the spread of step counts that the work estimate does not see.
    auto team_size = [&](int i, double M) {
      int T = (int)std::ceil(kTeamMargin * w[i] / M - 1e-9);
      T = std::min(T, maxT);
      return std::min(T, (b->h_inst[i].ns_a + 15) / 16);
    };
    const int budget = slots - slots / (cfg.queue_reserve == 0 ? kQueueReserve : cfg.queue_reserve);
    double M = std::max(total / slots, wmax / maxT);
    for (int it = 0; it < 200; ++it, M *= 1.05) {
      int used = 0;
      for (int i : by_work) {
        const int T = team_size(i, M);
        if (T < 2) break;
        used += T;
      }
      if (used <= budget) break;
    }
    std::vector<std::pair<int, int>> teams;  // (instance, members)
    int used = 0;
    for (int i : by_work) {
      const int T = team_size(i, M);
      if (T < 2 || used + T > budget) break;
      teams.push_back({i, T});
      used += T;
    }
    // The rounding of T leaves slots of the budget unused: give them one at
    // a time to the team with the most work per member.  On a tie the smaller
    // team gains (a 2-root team of 2 ties with a 3-root team of 3, and a
    // member added to the smaller team shortens it more).
    while (used < budget) {
      int best = -1;
      double bw = 0;
      for (int k = 0; k < (int)teams.size(); ++k) {
        const int i = teams[k].first, T = teams[k].second;
        if (T >= maxT || T >= (b->h_inst[i].ns_a + 15) / 16) continue;
        const double v = w[i] / T;
        if (best < 0 || v > bw * (1 + 1e-9) || (v > bw * (1 - 1e-9) && T < teams[best].second)) {
          bw = v;
          best = k;
        }
      }
      if (best < 0) break;
      teams[best].second += 1;
      used += 1;
    }
    for (const auto &t : teams) {
      for (int m = 0; m < t.second; ++m) blk.push_back(make_int4(t.first, t.second, m, pl.nteam));
      in_team[t.first] = 1;
      pl.nteam += 1;
    }
  }
  pl.ntw = (int)blk.size();
  std::vector<int> q;
  for (int i : (cfg.order == 0 ? by_work : ord))
    if (!in_team[i]) q.push_back(i);
  pl.nqueue = (int)q.size();
  pl.grid = std::max(1, std::max(pl.ntw, std::min(b->ncu * cfg.wg_per_cu, pl.ntw + pl.nqueue)));
  if (!q.empty())
    SBCI_HIP(hipMemcpyAsync(b->d_order, q.data(), sizeof(int) * q.size(), hipMemcpyHostToDevice,
                            b->stream));
  if (!blk.empty())
    SBCI_HIP(hipMemcpyAsync(b->d_team_blk, blk.data(), sizeof(int4) * blk.size(),
                            hipMemcpyHostToDevice, b->stream));
  // the host vectors must outlive the copies
  SBCI_HIP(hipStreamSynchronize(b->stream));
  return SBCI_OK;
}

int run_graph(sbci_batch *b, const sbci_batch_config &cfg, const BParams &P, double *ms,
              Plan *plan_out = nullptr) {
  size_t lds = 0;
  lds = lds_bytes(cfg.k_panel, cfg.threads);
  int resident = 0;
  if (cfg.threads == 256)
    SBCI_TRY(resident_blocks<256>(b, lds, &resident));
  else if (cfg.threads == 512)
    SBCI_TRY(resident_blocks<512>(b, lds, &resident));
  else
    SBCI_TRY(resident_blocks<1024>(b, lds, &resident));
  if (resident < 1) return batch_error(SBCI_EDEVICE, "batch kernel: no workgroup fits on a compute unit");
  Plan pl;
  SBCI_TRY(plan_launch(b, cfg, resident, pl));
  if (plan_out) *plan_out = pl;
  // The solve parameters are baked into the captured launch, so every call
  // captures a fresh graph (a few microseconds next to the solve).
  hipGraph_t g = nullptr;
  hipGraphExec_t x = nullptr;
  BParams Pc = P;
  Pc.kp = cfg.k_panel;
  Pc.team_wait = cfg.team_wait_us == 0 ? kTeamWaitTicks : (uint64_t)cfg.team_wait_us * kTicksPerUs;
  SBCI_HIP(hipMemcpyAsync(b->d_params, &Pc, sizeof(BParams), hipMemcpyHostToDevice, b->stream));
  int rc = SBCI_OK;
  if (cfg.threads == 256)
    rc = instantiate<256>(b, pl, lds, &x, &g);
  else if (cfg.threads == 512)
    rc = instantiate<512>(b, pl, lds, &x, &g);
  else
    rc = instantiate<1024>(b, pl, lds, &x, &g);
  if (rc != SBCI_OK) return rc;
  hipEvent_t e0, e1;
  SBCI_HIP(hipEventCreate(&e0));
  SBCI_HIP(hipEventCreate(&e1));
  SBCI_HIP(hipEventRecord(e0, b->stream));
  hipError_t e = hipGraphLaunch(x, b->stream);
  SBCI_HIP(hipEventRecord(e1, b->stream));
  hipError_t s = hipStreamSynchronize(b->stream);
  float t = 0;
  hipEventElapsedTime(&t, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipGraphExecDestroy(x);
  hipGraphDestroy(g);
  if (e != hipSuccess) return batch_error(SBCI_EDEVICE, std::string("graph launch: ") + hipGetErrorString(e));
  if (s != hipSuccess) return batch_error(SBCI_EDEVICE, std::string("batch solve: ") + hipGetErrorString(s));
  if (ms) *ms = t;
  return SBCI_OK;
}

sbci_batch_config default_config() {
  sbci_batch_config c{};
  c.threads = 256;
  c.wg_per_cu = 2;
  c.order = 0;
  c.k_panel = 16;
  c.max_team = 0;
  c.team_wait_us = 0;
  c.queue_reserve = 0;
  return c;
}

}  // namespace

extern "C" {

int sbci_batch_create(int ninst, const int *norb, const int *nalpha, const int *nbeta,
                      const double *const *h1, const double *const *eri, sbci_batch **out) {
  if (!out) return batch_error(SBCI_EINVAL, "out is NULL");
  *out = nullptr;
  if (ninst < 1) return batch_error(SBCI_EINVAL, "ninst must be >= 1");
  if (!norb || !nalpha || !nbeta || !h1 || !eri) return batch_error(SBCI_EINVAL, "NULL argument");
  for (int i = 0; i < ninst; ++i) {
    if (norb[i] < 1 || norb[i] > BMAX_NORB)
      return batch_error(SBCI_EINVAL, "batch instances need 1 <= norb <= 10");
    if (!h1[i] || !eri[i]) return batch_error(SBCI_EINVAL, "NULL integrals");
  }
  sbci_batch *b = new sbci_batch();
  b->ninst = ninst;
  hipError_t e = hipGetDevice(&b->device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, b->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete b;
    return batch_error(SBCI_EDEVICE, std::string("batch device setup: ") + hipGetErrorString(e));
  }
  b->ctx.assign(ninst, nullptr);
  b->la.resize(ninst);
  b->lb.resize(ninst);
  for (int i = 0; i < ninst; ++i) {
    int rc = create_context(norb[i], nalpha[i], nbeta[i], h1[i], eri[i], b->stream, false, &b->ctx[i]);
    if (rc == SBCI_OK) {
      sbci_ctx *c = b->ctx[i];
      if (c->A.ns > BMAX_NS || c->B.ns > BMAX_NS || c->A.s > BMAX_S || c->B.s > BMAX_S ||
          16 * ((c->npair + 15) / 16) > BMAX_NP)
        rc = batch_error(SBCI_EINVAL, "batch instance exceeds the workgroup limits");
    }
    if (rc == SBCI_OK) rc = build_dense(b, i);
    if (rc != SBCI_OK) {
      std::string m = sbci_last_error();
      sbci_batch_destroy(b);
      return batch_error(rc, "instance " + std::to_string(i) + ": " + m);
    }
  }
  hipError_t e2 = hipMalloc(&b->d_inst, sizeof(BInst) * ninst);
  if (e2 == hipSuccess) e2 = hipMalloc(&b->d_params, sizeof(BParams));
  if (e2 == hipSuccess) e2 = hipMalloc(&b->d_order, sizeof(int) * ninst);
  if (e2 == hipSuccess) e2 = hipMalloc(&b->d_queue, 256);
  if (e2 == hipSuccess) e2 = hipMalloc(&b->d_out, sizeof(BOut) * ninst);
  if (e2 == hipSuccess) e2 = hipMalloc(&b->d_team_blk, sizeof(int4) * (size_t)ninst * BMAX_TEAM);
  if (e2 == hipSuccess) e2 = hipMalloc(&b->d_tsync, sizeof(TeamSync) * (size_t)ninst);
  if (e2 == hipSuccess) e2 = hipStreamSynchronize(b->stream);
  if (e2 != hipSuccess) {
    sbci_batch_destroy(b);
    return batch_error(SBCI_EDEVICE, std::string("batch allocation: ") + hipGetErrorString(e2));
  }
  *out = b;
  return SBCI_OK;
}

int sbci_batch_destroy(sbci_batch *b) {
  if (!b) return SBCI_OK;
  if (b->stream) hipStreamSynchronize(b->stream);
  for (int i = 0; i < (int)b->ctx.size(); ++i) {
    const bool shared = b->ctx[i] && b->ctx[i]->B.shared;
    hipFree(b->la[i].d64);
    hipFree(b->la[i].d32);
    if (!shared) {
      hipFree(b->lb[i].d64);
      hipFree(b->lb[i].d32);
    }
    if (b->ctx[i]) sbci_destroy(b->ctx[i]);
  }
  hipFree(b->d_inst);
  hipFree(b->d_params);
  hipFree(b->d_order);
  hipFree(b->d_queue);
  hipFree(b->d_out);
  hipFree(b->d_team_blk);
  hipFree(b->d_tsync);
  hipFree(b->arena64);
  hipFree(b->arena32);
  if (b->stream) hipStreamDestroy(b->stream);
  delete b;
  return SBCI_OK;
}

int64_t sbci_batch_ndet(const sbci_batch *b, int inst) {
  if (!b || inst < 0 || inst >= b->ninst) return -1;
  return b->ctx[inst]->ndet;
}

int sbci_batch_solve(sbci_batch *b, const int *nroots, double tol, const sbci_opts *opt,
                     const sbci_batch_config *cfg_in, double *energies, sbci_batch_inst *info,
                     sbci_batch_report *rep) {
  if (!b || !nroots) return batch_error(SBCI_EINVAL, "NULL argument");
  BParams P{};
  int precision = 0;
  SBCI_TRY(params_from(opt, tol, P, precision));
  sbci_batch_config cfg = cfg_in ? *cfg_in : (b->have_tuned ? b->tuned : default_config());
  SBCI_TRY(check_config(cfg));
  SBCI_TRY(prepare(b, nroots, precision));
  double ms = 0;
  Plan pl;
  SBCI_TRY(run_graph(b, cfg, P, &ms, &pl));
  b->solved_precision = precision;
  std::vector<BOut> o(b->ninst);
  SBCI_HIP(hipMemcpy(o.data(), b->d_out, sizeof(BOut) * b->ninst, hipMemcpyDeviceToHost));
  sbci_batch_report r{};
  r.seconds = ms * 1e-3;
  uint64_t tmin = ~0ull, tmax = 0;
  for (const BOut &q : o) {
    tmin = std::min(tmin, q.t0);
    tmax = std::max(tmax, q.t1);
  }
  int64_t off = 0;
  int worst = SBCI_OK;
  for (int i = 0; i < b->ninst; ++i) {
    const BOut &q = o[i];
    for (int a = 0; a < nroots[i]; ++a) {
      if (energies) energies[off + a] = a < q.nconv ? q.E[a] : NAN;
    }
    off += nroots[i];
    if (info) {
      sbci_batch_inst &f = info[i];
      f.status = q.status;
      f.nroots_converged = q.nconv;
      f.nsteps = q.nsteps;
      f.nrestarts = q.nrestarts;
      f.nsigma_f64 = q.nsig64;
      f.nsigma_low = q.nsiglow;
      f.t_start = (double)(q.t0 - tmin) / kRealtimeHz;
      f.t_end = (double)(q.t1 - tmin) / kRealtimeHz;
      for (int a = 0; a < 4; ++a) f.resid[a] = a < q.nconv ? q.dz[a] : NAN;
      f.t_same = (double)q.tsig[0] / kRealtimeHz;
      f.t_opp = (double)q.tsig[1] / kRealtimeHz;
    }
    if (q.status == SBCI_OK) r.ninst_converged += 1;
    else if (worst == SBCI_OK || q.status == SBCI_ENUMERIC || q.status == SBCI_EDEVICE) worst = q.status;
    if (q.status == SBCI_EDEVICE) r.team_timeouts += 1;
    r.nsigma_f64 += q.nsig64;
    r.nsigma_low += q.nsiglow;
    r.det_sigma += (int64_t)b->ctx[i]->ndet * (q.nsig64 + q.nsiglow);
    r.nsteps += q.nsteps;
    r.nrestarts += q.nrestarts;
  }
  r.span_seconds = tmax > tmin ? (double)(tmax - tmin) / kRealtimeHz : 0.0;
  r.threads = cfg.threads;
  r.wg_per_cu = cfg.wg_per_cu;
  r.order = cfg.order;
  r.k_panel = cfg.k_panel;
  r.max_team = cfg.max_team;
  r.team_wait_us = cfg.team_wait_us;
  r.queue_reserve = cfg.queue_reserve;
  r.nteams = pl.nteam;
  r.team_workgroups = pl.ntw;
  if (rep) *rep = r;
  if (worst != SBCI_OK)
    return batch_error(worst, worst == SBCI_ENOCONV   ? "some batch instances did not converge"
                              : worst == SBCI_EDEVICE ? "a team of workgroups exceeded its wait bound"
                                                      : "numerical failure in a batch instance");
  return SBCI_OK;
}

int sbci_batch_tune(sbci_batch *b, const int *nroots, double tol, const sbci_opts *opt,
                    sbci_batch_config *best, double *ms_out, sbci_batch_config *cand_out,
                    int *ncand) {
  if (!b || !nroots) return batch_error(SBCI_EINVAL, "NULL argument");
  BParams P{};
  int precision = 0;
  SBCI_TRY(params_from(opt, tol, P, precision));
  SBCI_TRY(prepare(b, nroots, precision));
  // stage 1: workgroup size x residency (longest-first, tall tiles);
  // stage 2: queue order, tile height and queue reserve around the winner.
  std::vector<sbci_batch_config> tried;
  std::vector<double> times;
  auto trial = [&](const sbci_batch_config &c) -> int {
    double ms = 0;
    SBCI_TRY(run_graph(b, c, P, &ms));
    tried.push_back(c);
    times.push_back(ms);
    return SBCI_OK;
  };
  for (int nt : {256, 512, 1024})
    for (int w : {1, 2}) {
      sbci_batch_config c{};
      c.threads = nt;
      c.wg_per_cu = w;
      c.order = 0;
      c.k_panel = 16;
      c.max_team = 0;
      SBCI_TRY(trial(c));
    }
  size_t bi = std::min_element(times.begin(), times.end()) - times.begin();
  sbci_batch_config w = tried[bi];
  {
    sbci_batch_config c = w;
    c.order = 1;
    SBCI_TRY(trial(c));
    c = w;
    c.k_panel = 8;
    SBCI_TRY(trial(c));
    c = w;
    c.queue_reserve = 8;
    SBCI_TRY(trial(c));
  }
  bi = std::min_element(times.begin(), times.end()) - times.begin();
  b->tuned = tried[bi];
  b->have_tuned = true;
  if (best) *best = tried[bi];
  const int n = (int)tried.size();
  if (ncand) {
    const int cap = *ncand;
    for (int i = 0; i < n && i < cap; ++i) {
      if (ms_out) ms_out[i] = times[i];
      if (cand_out) cand_out[i] = tried[i];
    }
    *ncand = n;
  }
  return SBCI_OK;
}

int sbci_batch_vectors(sbci_batch *b, int inst, double *dev_out) {
  if (!b || !dev_out || inst < 0 || inst >= b->ninst) return batch_error(SBCI_EINVAL, "bad argument");
  if (b->h_inst.empty()) return batch_error(SBCI_EINVAL, "sbci_batch_vectors before a solve");
  const BInst &I = b->h_inst[inst];
  BOut o;
  SBCI_HIP(hipMemcpy(&o, b->d_out + inst, sizeof(BOut), hipMemcpyDeviceToHost));
  const int nc = std::min(o.nconv, I.nroots);
  SBCI_HIP(hipMemcpyAsync(dev_out, I.v64 + (int64_t)NVW * I.ndet, sizeof(double) * I.ndet * nc,
                          hipMemcpyDeviceToDevice, b->stream));
  SBCI_HIP(hipStreamSynchronize(b->stream));
  return SBCI_OK;
}

}  // extern "C"
