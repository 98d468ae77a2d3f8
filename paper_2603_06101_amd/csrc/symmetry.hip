// Point-group symmetry blocking: sigma on the determinants of one irrep.
//
// Every molecule of the paper is solved inside one irreducible
// representation of its point group (the IRep column of the Section S3.1
// table, whose determinant counts are the full C(norb, na) * C(norb, nb)
// products, not the size of that irrep's block).  For an abelian
// group with irreps 0..7 that multiply by XOR (D2h and its subgroups), a
// string's irrep is the XOR of its occupied orbitals' irreps and |Ia, Ib> has
// irrep irr(Ia) ^ irr(Ib).  Totally symmetric integrals make H block
// diagonal, so the states of irrep G live on
//   block a = 0..7:  [alpha strings of irrep a] x [beta strings of irrep a ^ G]
// stored row-major, blocks one after another.  Within a block strings keep
// their ascending-mask order; pos[I] is a string's rank inside its irrep.
//
// sigma on that layout (no full-space vector is ever formed):
//   same-spin  sigma[a](r, q) = sum_g Fb[Ib][g] c[a](r, posB[J_g])
//                             + sum_g Fa[Ia][g] c[a](posA[J_g], q)
//              over the same-spin lists compacted to entries inside the
//              string's own irrep (the others are exactly zero);
//   opposite   sigma[a](r, q) += sum_f sign_f sum_{e: cls(e) = cls(f)}
//              (pq_e|rs_f) sign_e c[a ^ cls](posA[J_e], posB[J_f])
//              over the single-excitation tables of Ia (e) and Ib (f), where
//              cls(E_pq) = orbsym[p] ^ orbsym[q]; the integral vanishes when
//              the classes differ, and when they agree the source
//              determinant lies in block a ^ cls.
// Kernels: the beta same-spin part is an in-row gather over transposed lists,
// from rows staged in LDS (k_sym_same_lds; k_sym_same gathers from global
// memory where the rows are too long); the alpha same-spin part runs block by block through the
// list kernel of the unblocked sigma; the opposite-spin part is the pair form
// (k_sym_opp_pair: one alpha string per workgroup, the row of sigma and the
// class blocks of integrals in LDS), or the gather form (k_sym_opp) where that
// does not fit in LDS.  In FP64 the pair and MFMA forms scatter in 64-bit
// fixed point as the unblocked sigma does (k_sym_rowmax gives each row's
// scale), so the blocked FP64 sigma too is the same to the last bit from call
// to call; the gather form sums each output in a fixed order.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"
#include "mfma.h"

namespace sbci {

namespace {

// Block geometry passed by value to the kernels.
struct SymArgs {
  int64_t off[9];     // block offsets in a vector (off[8] = ndet)
  int64_t rowsA[8];   // alpha strings of irrep a
  int64_t ncol[8];    // beta strings of irrep a ^ G (block a's row length)
  int64_t startA[9];  // first irrep-sorted alpha index of irrep a
  int64_t startBc[8]; // first irrep-sorted beta index of irrep a ^ G
};

__device__ __forceinline__ int find_block(const SymArgs &g, int64_t d) {
  int a = 0;
#pragma unroll
  for (int k = 1; k < 8; ++k)
    if (g.off[k] <= d) a = k;
  return a;
}

// Keep the same-spin list entries whose target lies in the row string's
// irrep, as (rank inside the irrep, value); pad with (own rank, 0).
__global__ void k_sym_count(const int32_t *__restrict__ fcol, int nf, int64_t ns,
                            const int32_t *__restrict__ irr, int32_t *__restrict__ cnt) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= ns) return;
  int k = 0;
  for (int e = 0; e < nf; ++e) k += irr[fcol[i * nf + e]] == irr[i];
  cnt[i] = k;
}

// The compacted lists with rows in irrep-sorted order (start: first sorted
// index of each irrep), row-major [sorted string][entry] or transposed
// [entry][sorted string] (the lanes of a wave, which own consecutive strings of
// one irrep, then read them coalesced).
__global__ void k_sym_compact(const int32_t *__restrict__ fcol, const double *__restrict__ f64,
                              int nf, int64_t ns, const int32_t *__restrict__ irr,
                              const int32_t *__restrict__ pos, int nfs,
                              const int64_t *__restrict__ start, int transposed,
                              int32_t *__restrict__ col, double *__restrict__ v64,
                              float *__restrict__ v32) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= ns) return;
  const int64_t is = start[irr[i]] + pos[i];
  int k = 0;
  for (int e = 0; e < nf; ++e) {
    const int32_t J = fcol[i * nf + e];
    if (irr[J] != irr[i]) continue;
    const int64_t o = transposed ? (int64_t)k * ns + is : is * nfs + k;
    col[o] = pos[J];
    v64[o] = f64[i * nf + e];
    v32[o] = (float)f64[i * nf + e];
    ++k;
  }
  for (; k < nfs; ++k) {
    const int64_t o = transposed ? (int64_t)k * ns + is : is * nfs + k;
    col[o] = pos[i];
    v64[o] = 0.0;
    v32[o] = 0.0f;
  }
}

// Blocked copy of a full-space array (the diagonal): one blocked element per thread.
template <typename T>
__global__ void k_sym_gather(SymArgs g, const int32_t *__restrict__ idxA,
                             const int32_t *__restrict__ idxB, int64_t nsb,
                             const T *__restrict__ full, T *__restrict__ out) {
  const int64_t nd = g.off[8];
  for (int64_t d = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; d < nd;
       d += (int64_t)gridDim.x * blockDim.x) {
    const int a = find_block(g, d);
    const int64_t nc = g.ncol[a], rel = d - g.off[a];
    const int64_t r = rel / nc, q = rel - r * nc;
    const int64_t Ia = idxA[g.startA[a] + r], Ib = idxB[g.startBc[a] + q];
    out[d] = full[Ia * nsb + Ib];
  }
}

// Beta same-spin part (with the beta one-electron terms), plain write; the
// alpha part follows block by block with the list kernel of the unblocked
// sigma.  In-row gathers over the transposed lists: the list
// of column q (beta string Ib) is the same for every row of the block, so a
// thread takes one column and kSymSameRows rows: each list entry is loaded
// once for the group (coalesced over q) and gathered from each row.  Work
// items: block a holds ceil(rows_a / kSymSameRows) x ncol[a] of them, from
// rg.off[a] on.
constexpr int kSymSameRows = 8;
struct RowGroups {
  int64_t off[9];
};
// LDS form of the beta gathers: rows per workgroup and the LDS it may take
constexpr int kSymSameLdsRows = 4;
constexpr size_t kSymSameLdsMax = 160 * 1024 / 3;  // three workgroups per CU

template <typename T, typename V>
__global__ __launch_bounds__(256) void k_sym_same(
    SymArgs g, RowGroups rg, const int32_t *__restrict__ colBT, const V *__restrict__ valBT,
    int nfB, int64_t nsb, const T *__restrict__ c, T *__restrict__ out) {
  const int64_t d = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (d >= rg.off[8]) return;
  int a = 0;
#pragma unroll
  for (int k = 1; k < 8; ++k)
    if (rg.off[k] <= d) a = k;
  const int64_t vo = (int64_t)blockIdx.y * g.off[8];
  const int64_t nc = g.ncol[a], rel = d - rg.off[a];
  const int64_t grp = rel / nc, q = rel - grp * nc;
  const int64_t r0 = grp * kSymSameRows;
  const int nr = (int)(g.rowsA[a] - r0 < kSymSameRows ? g.rowsA[a] - r0 : kSymSameRows);
  const int64_t qs = g.startBc[a] + q;
  const T *__restrict__ blk = c + vo + g.off[a] + r0 * nc;
  T acc[kSymSameRows];
#pragma unroll
  for (int i = 0; i < kSymSameRows; ++i) acc[i] = 0;
  for (int e = 0; e < nfB; ++e) {
    const T v = (T)valBT[(int64_t)e * nsb + qs];
    const int64_t col = colBT[(int64_t)e * nsb + qs];
#pragma unroll
    for (int i = 0; i < kSymSameRows; ++i)
      if (i < nr) acc[i] += v * blk[i * nc + col];
  }
  T *__restrict__ o = out + vo + g.off[a] + r0 * nc + q;
#pragma unroll
  for (int i = 0; i < kSymSameRows; ++i)
    if (i < nr) o[i * nc] = acc[i];
}

// The same beta gathers with the rows in LDS: one workgroup per group of
// RG rows of a block (the groups of block a start at rg.off[a]); the group's
// rows (contiguous in the block, RG x ncol[a] elements) are staged once, and
// each thread walks the lists of its columns, gathering from LDS.  Random
// columns of a global row touch up to 64 cache lines per wave instruction;
// from LDS they cost bank cycles only.
template <typename T, typename V, int RG>
__global__ __launch_bounds__(256) void k_sym_same_lds(
    SymArgs g, RowGroups rg, const int32_t *__restrict__ colBT, const V *__restrict__ valBT,
    int nfB, int64_t nsb, const T *__restrict__ c, T *__restrict__ out) {
  extern __shared__ __align__(16) unsigned char smem[];
  T *L = reinterpret_cast<T *>(smem);  // [RG][nc]
  const int64_t k = blockIdx.x;
  int a = 0;
#pragma unroll
  for (int t = 1; t < 8; ++t)
    if (rg.off[t] <= k) a = t;
  const int64_t nc = g.ncol[a];
  const int64_t r0 = (k - rg.off[a]) * RG;
  const int nr = (int)(g.rowsA[a] - r0 < RG ? g.rowsA[a] - r0 : RG);
  const int64_t vo = (int64_t)blockIdx.y * g.off[8];
  const T *__restrict__ blk = c + vo + g.off[a] + r0 * nc;
  for (int64_t i = threadIdx.x; i < nr * nc; i += 256) L[i] = blk[i];
  __syncthreads();
  T *__restrict__ o = out + vo + g.off[a] + r0 * nc;
  for (int64_t q = threadIdx.x; q < nc; q += 256) {
    const int64_t qs = g.startBc[a] + q;
    T acc[RG];
#pragma unroll
    for (int i = 0; i < RG; ++i) acc[i] = 0;
    for (int e = 0; e < nfB; ++e) {
      const T v = (T)valBT[(int64_t)e * nsb + qs];
      const int col = colBT[(int64_t)e * nsb + qs];
#pragma unroll
      for (int i = 0; i < RG; ++i)
        if (i < nr) acc[i] += v * L[i * nc + col];
    }
#pragma unroll
    for (int i = 0; i < RG; ++i)
      if (i < nr) o[i * nc + q] = acc[i];
  }
}

// Opposite-spin part in gather form (used where the pair form below does not
// fit in LDS), accumulated: one workgroup per alpha string (irrep-sorted
// index k), threads over the row's beta columns.
// LDS: srcoff[sA] (int64, source row offset in the vector) | wro[sA] (int32,
// pair row of W) | ord[sA] (class-sorted entry) | cls[sA] | cs[9] | sg[sA] (T, sign).
template <typename T>
__global__ __launch_bounds__(256) void k_sym_opp(
    SymArgs g, const int32_t *__restrict__ orbsym, const int32_t *__restrict__ idxA,
    const int32_t *__restrict__ idxB, const int32_t *__restrict__ posA,
    const int32_t *__restrict__ posB, const Ent *__restrict__ tabA, int sA,
    const Ent *__restrict__ tabB, int sB, const T *__restrict__ W, int npair,
    const T *__restrict__ c, T *__restrict__ out) {
  extern __shared__ __align__(16) unsigned char smem[];
  int64_t *srcoff = reinterpret_cast<int64_t *>(smem);
  int32_t *wro = reinterpret_cast<int32_t *>(srcoff + sA);
  int32_t *ord = wro + sA;
  int32_t *cls = ord + sA;
  int32_t *cs = cls + sA;  // [9]
  T *sg = reinterpret_cast<T *>(smem + (((size_t)sA * 20 + 36 + 15) & ~(size_t)15));
  const int64_t k = blockIdx.x;
  int a = 0;
#pragma unroll
  for (int t = 1; t < 8; ++t)
    if (g.startA[t] <= k) a = t;
  const int64_t nc = g.ncol[a];
  if (nc == 0) return;  // uniform over the workgroup
  const int64_t r = k - g.startA[a];
  const int64_t Ia = idxA[k];
  const int64_t nd = g.off[8];
  const int64_t vo = (int64_t)blockIdx.y * nd;
  for (int e = threadIdx.x; e < sA; e += blockDim.x) {
    const Ent t = tabA[Ia * sA + e];
    const int x = orbsym[t.p] ^ orbsym[t.q];
    const int b = a ^ x;  // block of the source determinants
    cls[e] = x;
    srcoff[e] = g.off[b] + (int64_t)posA[t.J] * g.ncol[b];
    wro[e] = pair_index(t.p, t.q) * npair;
    sg[e] = (T)t.sign;
  }
  __syncthreads();
  if (threadIdx.x == 0) {  // counting sort of the entries by class
    int n[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int e = 0; e < sA; ++e) ++n[cls[e]];
    cs[0] = 0;
    for (int x = 0; x < 8; ++x) cs[x + 1] = cs[x] + n[x];
    int fill[8];
    for (int x = 0; x < 8; ++x) fill[x] = cs[x];
    for (int e = 0; e < sA; ++e) ord[fill[cls[e]]++] = e;
  }
  __syncthreads();
  const T *__restrict__ cv = c + vo;
  T *__restrict__ row = out + vo + g.off[a] + r * nc;
  for (int64_t q = threadIdx.x; q < nc; q += blockDim.x) {
    const int64_t Ib = idxB[g.startBc[a] + q];
    T acc = 0;
    for (int f = 0; f < sB; ++f) {
      const Ent t = tabB[Ib * sB + f];
      const int x = orbsym[t.p] ^ orbsym[t.q];
      const int kl = pair_index(t.p, t.q);
      const int64_t jp = posB[t.J];
      T inner = 0;
      for (int i = cs[x]; i < cs[x + 1]; ++i) {
        const int e = ord[i];
        inner += sg[e] * W[wro[e] + kl] * cv[srcoff[e] + jp];
      }
      acc += (T)t.sign * inner;
    }
    row[q] += acc;
  }
}

// max |c| of every block row (irrep-sorted alpha index k, vector blockIdx.y):
// the fixed-point scale of the FP64 opposite-spin scatter; NaN if the row
// holds a NaN
__global__ __launch_bounds__(256) void k_sym_rowmax(SymArgs g, const double *__restrict__ c,
                                                    int64_t nsa, double *__restrict__ out) {
  __shared__ double red[4];
  const int64_t k = blockIdx.x;
  int a = 0;
#pragma unroll
  for (int t = 1; t < 8; ++t)
    if (g.startA[t] <= k) a = t;
  const int64_t n = g.ncol[a];
  const double *row = c + (int64_t)blockIdx.y * g.off[8] + g.off[a] + (k - g.startA[a]) * n;
  double m = 0.0;
  for (int64_t j = threadIdx.x; j < n; j += 256) {
    const double v = fabs(row[j]);
    m = (v > m || v != v) ? v : m;
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
    out[(int64_t)blockIdx.y * nsa + k] = r;
  }
}

// Largest (NaN-propagating) m over a 256-thread workgroup; every thread
// calls it (it holds a barrier) and receives the result.
__device__ inline double wg_max256(double m, double *red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double r = __shfl_xor(m, o);
    m = (r > m || r != r) ? r : m;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  m = 0.0;
#pragma unroll
  for (int w = 0; w < 4; ++w) m = (red[w] > m || red[w] != red[w]) ? red[w] : m;
  return m;
}

// Dynamic LDS of the blocked opposite-spin kernels: a CU's 160 KB less the
// static slots of the fixed-point scale reduction.
constexpr size_t kSymLdsCap = 160 * 1024 - 256;

// Pair form of the opposite-spin part: one workgroup per alpha string Ia
// (irrep-sorted index k, block a), the row of sigma accumulated in LDS.  For
// each class x with alpha excitations e of Ia, the source block is a ^ x and
// for each of its columns J (a beta string) and each orbital pair kl of class x
//   M[kl][J] = sum_e sign_e (kl_e|kl) c[a ^ x](rank(J_e), J)
// is formed in registers (8 pairs at a time) and scattered through the beta
// pair code of (kl, J) to the row entry of E_kl J or E_lk J (the one that is
// not zero), with that sign.  c is read along rows (coalesced), W from LDS:
// class x's integrals sign_e (kl_e|kl) are a K_x x P8_x block (rows padded
// with zeros to whole tiles of 8 pairs), so a tile's 8 values are contiguous.
// LDS: acc[maxcol] (double) | srcoff, wro, ord, cls, cs[9], woff[9] | sg | so2
//      | Ws[<= sA * maxp8] | plist[npair]   (maxp8: the largest class, padded to 8)
// FIX (FP64): acc holds 64-bit fixed point; the row's scale comes from the
// largest |c| over the source rows its excitations gather (rowmax) times
// wbound, a bound on every partial sum of a row per unit of |c| (as in the
// unblocked sigma; the blocked sums are a subset of its terms).
struct PairStarts {
  int s[9];
};

template <typename T, bool FIXT>
__global__ __launch_bounds__(256) void k_sym_opp_pair(
    SymArgs g, PairStarts pcs, const int32_t *__restrict__ orbsym, const int32_t *__restrict__ idxA,
    const int32_t *__restrict__ posA, const Ent *__restrict__ tabA, int sA,
    const uint32_t *__restrict__ pairS, int64_t nsb, const int32_t *__restrict__ plist_g,
    const T *__restrict__ W, int npair, int64_t maxcol, int maxp8, const T *__restrict__ c,
    T *__restrict__ out, const double *__restrict__ rowmax, double wbound) {
  constexpr bool FIX = FIXT && std::is_same<T, double>::value;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double wmax[4];
  double *acc = reinterpret_cast<double *>(smem);
  unsigned char *base = smem + (((size_t)maxcol * 8 + 15) & ~(size_t)15);
  int64_t *srcoff = reinterpret_cast<int64_t *>(base);
  int32_t *wro = reinterpret_cast<int32_t *>(srcoff + sA);
  int32_t *ord = wro + sA;
  int32_t *cls = ord + sA;
  int32_t *cs = cls + sA;  // [9]
  int32_t *woff = cs + 9;  // [9]
  const size_t o1 = ((size_t)sA * 20 + 72 + 15) & ~(size_t)15;
  T *sg = reinterpret_cast<T *>(base + o1);
  const size_t o2 = (o1 + (size_t)sA * sizeof(T) + 7) & ~(size_t)7;
  int64_t *so2 = reinterpret_cast<int64_t *>(base + o2);
  const size_t ow = (o2 + (size_t)sA * 8 + 15) & ~(size_t)15;
  T *Ws = reinterpret_cast<T *>(base + ow);
  int32_t *plist = reinterpret_cast<int32_t *>(Ws + (size_t)sA * maxp8);

  const int64_t k = blockIdx.x;
  int a = 0;
#pragma unroll
  for (int t = 1; t < 8; ++t)
    if (g.startA[t] <= k) a = t;
  const int64_t nc = g.ncol[a];
  if (nc == 0) return;  // uniform over the workgroup
  const int64_t r = k - g.startA[a];
  const int64_t Ia = idxA[k];
  const int64_t vo = (int64_t)blockIdx.y * g.off[8];
  for (int64_t j = threadIdx.x; j < nc; j += blockDim.x) acc[j] = 0.0;
  double rm = 0.0;
  for (int e = threadIdx.x; e < sA; e += blockDim.x) {
    const Ent t = tabA[Ia * sA + e];
    const int x = orbsym[t.p] ^ orbsym[t.q];
    const int b = a ^ x;
    cls[e] = x;
    srcoff[e] = g.off[b] + (int64_t)posA[t.J] * g.ncol[b];
    wro[e] = pair_index(t.p, t.q) * npair;
    sg[e] = (T)t.sign;
    if constexpr (FIX) {
      const double v = rowmax[(int64_t)blockIdx.y * g.startA[8] + g.startA[b] + posA[t.J]];
      rm = (v > rm || v != v) ? v : rm;
    }
  }
  for (int p = threadIdx.x; p < npair; p += blockDim.x) plist[p] = plist_g[p];
  double fscale = 1.0, finv = 1.0;
  bool fbad = false;
  if constexpr (FIX) fix_scale_from_bound(wbound * wg_max256(rm, wmax), fscale, finv, fbad);
  __syncthreads();
  if (threadIdx.x == 0) {
    int n[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int e = 0; e < sA; ++e) ++n[cls[e]];
    cs[0] = 0;
    for (int x = 0; x < 8; ++x) cs[x + 1] = cs[x] + n[x];
    int fill[8];
    for (int x = 0; x < 8; ++x) fill[x] = cs[x];
    for (int e = 0; e < sA; ++e) ord[fill[cls[e]]++] = e;
    woff[0] = 0;
    for (int x = 0; x < 8; ++x)
      woff[x + 1] = woff[x] + n[x] * ((pcs.s[x + 1] - pcs.s[x] + 7) & ~7);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < sA; i += blockDim.x) so2[i] = srcoff[ord[i]];
  for (int x = 0; x < 8; ++x) {
    const int np_ = pcs.s[x + 1] - pcs.s[x], p8 = (np_ + 7) & ~7;
    const int nx = (cs[x + 1] - cs[x]) * p8;
    for (int y = threadIdx.x; y < nx; y += blockDim.x) {
      const int il = y / p8, pl = y - il * p8;
      const int e = ord[cs[x] + il];
      // FIX: the power-of-two scale folded in (exact); M comes out in fixed-point units
      Ws[woff[x] + y] = pl < np_ ? sg[e] * W[wro[e] + plist[pcs.s[x] + pl]] * (T)fscale : (T)0;
    }
  }
  __syncthreads();
  const T *__restrict__ cv = c + vo;
  for (int x = 0; x < 8; ++x) {
    const int i0 = cs[x], i1 = cs[x + 1];
    const int p0 = pcs.s[x], p1 = pcs.s[x + 1];
    if (i0 == i1 || p0 == p1) continue;  // uniform
    const int b = a ^ x;
    const int64_t nbc = g.ncol[b];
    const int64_t col0 = g.startBc[b];  // irrep-sorted beta index of column 0 of block b
    const int p8 = (p1 - p0 + 7) & ~7;
    const T *__restrict__ wc = Ws + woff[x];
    for (int64_t j = threadIdx.x; j < nbc; j += blockDim.x) {
      for (int pp = p0; pp < p1; pp += 8) {
        int kl[8];
        T m[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          kl[t] = plist[pp + t < p1 ? pp + t : p0];
          m[t] = 0;
        }
        const T *__restrict__ wt = wc + (pp - p0);
        for (int i = i0; i < i1; ++i) {
          const T v = cv[so2[i] + j];
          const T *wr = wt + (size_t)(i - i0) * p8;
#pragma unroll
          for (int t = 0; t < 8; ++t) m[t] += wr[t] * v;
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          if (pp + t < p1) {
            const uint32_t cd = pairS[(int64_t)kl[t] * nsb + col0 + j];
            if (cd != kInvalid) {
              const double v = (double)m[t];
              scatter_add<FIX>(&acc[cd >> 1], (cd & 1u) ? -v : v);
            }
          }
        }
      }
    }
  }
  __syncthreads();
  T *__restrict__ row = out + vo + g.off[a] + r * nc;
  for (int64_t j = threadIdx.x; j < nc; j += blockDim.x) row[j] += row_value<FIX, T>(acc, j, finv, fbad);
}

// MFMA form of the pair contraction above, the same sums: for each class x
// with alpha excitations e of Ia and pairs kl of class x, the product
//   M[kl][J] = sum_e A_x[kl][e] c[a ^ x](rank(J_e), J),
//   A_x[kl][e] = sign_e (kl_e|kl)
// runs as 16 x 16 MFMA tiles: A_x (its pairs padded to whole 16-row tiles,
// its excitations to whole k-steps, zeros in the padding) sits in LDS, and
// each wave takes 16-column tiles J of the source block, gathers the B
// fragments c[a ^ x](rank(J_e), J) from the vector and scatters M through
// the beta pair codes, as the pair form does.  Flavour M: FP64, FP32, or BF16
// operands with FP32 accumulation (T = float).  Classes with more than
// kSymMmaRows pairs use the pair form.
// LDS: acc[maxcol] (double) | A tile [kSymMmaRows][lda] (16-byte aligned)
//      | so2[sA] (uint32) | ord, cls[sA] | cs[9] | wro[sA] | sg[sA] (double)
//      | plist[npair] | srcoff[sA] (uint32)
constexpr int kSymMmaRows = 64;

template <typename M, typename T, bool FIXT>
__global__ __launch_bounds__(256) void k_sym_opp_mma(
    SymArgs g, PairStarts pcs, const int32_t *__restrict__ orbsym, const int32_t *__restrict__ idxA,
    const int32_t *__restrict__ posA, const Ent *__restrict__ tabA, int sA,
    const uint32_t *__restrict__ pairS, int64_t nsb, const int32_t *__restrict__ plist_g,
    const T *__restrict__ W, int npair, int64_t maxcol, const T *__restrict__ c, T *__restrict__ out,
    const double *__restrict__ rowmax, double wbound) {
  // FIX (FP64): fixed-point scatter, as in the pair form
  constexpr bool FIX = FIXT && std::is_same<M, MF64>::value;
  __shared__ double wmax[4];
  using A = typename M::A;
  using Frag = typename M::Frag;
  using Out = typename M::Out;
  constexpr int NW = 4;
  constexpr int MTMAX = kSymMmaRows / 16;
  extern __shared__ __align__(16) unsigned char smem[];
  const int ksmax = (sA + M::KSTEP - 1) / M::KSTEP;
  const int lda = ksmax * M::KSTEP + M::PAD;
  double *acc = reinterpret_cast<double *>(smem);
  A *At = reinterpret_cast<A *>(smem + (((size_t)maxcol * 8 + 15) & ~(size_t)15));
  unsigned char *base = reinterpret_cast<unsigned char *>(At) +
                        ((((size_t)kSymMmaRows * lda * sizeof(A)) + 15) & ~(size_t)15);
  uint32_t *so2 = reinterpret_cast<uint32_t *>(base);
  int32_t *ord = reinterpret_cast<int32_t *>(so2 + sA);
  int32_t *cls = ord + sA;
  int32_t *cs = cls + sA;  // [9]
  int32_t *wro = cs + 9;
  double *sg = reinterpret_cast<double *>(base + ((((size_t)sA * 16 + 36) + 15) & ~(size_t)15));
  int32_t *plist = reinterpret_cast<int32_t *>(sg + sA);
  uint32_t *srcoff = reinterpret_cast<uint32_t *>(plist + npair);

  const int64_t k = blockIdx.x;
  int a = 0;
#pragma unroll
  for (int t = 1; t < 8; ++t)
    if (g.startA[t] <= k) a = t;
  const int64_t nc = g.ncol[a];
  if (nc == 0) return;  // uniform over the workgroup
  const int64_t r = k - g.startA[a];
  const int64_t Ia = idxA[k];
  const int64_t vo = (int64_t)blockIdx.y * g.off[8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, li = lane & 15, gq = lane >> 4;
  for (int64_t j = tid; j < nc; j += 64 * NW) acc[j] = 0.0;
  double rm = 0.0;
  for (int e = tid; e < sA; e += 64 * NW) {
    const Ent t = tabA[Ia * sA + e];
    const int x = orbsym[t.p] ^ orbsym[t.q];
    const int b = a ^ x;
    cls[e] = x;
    srcoff[e] = (uint32_t)(g.off[b] + (int64_t)posA[t.J] * g.ncol[b]);
    wro[e] = pair_index(t.p, t.q) * npair;
    sg[e] = (double)t.sign;
    if constexpr (FIX) {
      const double v = rowmax[(int64_t)blockIdx.y * g.startA[8] + g.startA[b] + posA[t.J]];
      rm = (v > rm || v != v) ? v : rm;
    }
  }
  for (int p = tid; p < npair; p += 64 * NW) plist[p] = plist_g[p];
  double fscale = 1.0, finv = 1.0;
  bool fbad = false;
  if constexpr (FIX) fix_scale_from_bound(wbound * wg_max256(rm, wmax), fscale, finv, fbad);
  __syncthreads();
  if (tid == 0) {
    int n[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int e = 0; e < sA; ++e) ++n[cls[e]];
    cs[0] = 0;
    for (int x = 0; x < 8; ++x) cs[x + 1] = cs[x] + n[x];
    int fill[8];
    for (int x = 0; x < 8; ++x) fill[x] = cs[x];
    for (int e = 0; e < sA; ++e) ord[fill[cls[e]]++] = e;
  }
  __syncthreads();
  for (int i = tid; i < sA; i += 64 * NW) so2[i] = srcoff[ord[i]];
  __syncthreads();
  const T *__restrict__ cv = c + vo;
  for (int x = 0; x < 8; ++x) {
    const int i0 = cs[x], nx = cs[x + 1] - cs[x];
    const int p0 = pcs.s[x], np_ = pcs.s[x + 1] - pcs.s[x];
    if (nx == 0 || np_ == 0) continue;  // uniform
    const int b = a ^ x;
    const int64_t nbc = g.ncol[b];
    const int64_t col0 = g.startBc[b];
    const int mt = (np_ + 15) / 16;   // <= MTMAX (checked on the host)
    const int ks = (nx + M::KSTEP - 1) / M::KSTEP;
    // A_x: rows = pairs of class x, columns = its excitations (class order)
    for (int y = tid; y < mt * 16 * ks * M::KSTEP; y += 64 * NW) {
      const int row = y / (ks * M::KSTEP), kk = y - row * (ks * M::KSTEP);
      double v = 0.0;
      if (row < np_ && kk < nx) {
        const int e = ord[i0 + kk];
        v = sg[e] * (double)W[wro[e] + plist[p0 + row]] * fscale;  // FIX: exact power of two
      }
      At[row * lda + kk] = M::cvt(v);
    }
    __syncthreads();
    const int njt = (int)((nbc + 15) / 16);
    for (int jt = wave; jt < njt; jt += NW) {
      const int64_t col = (int64_t)jt * 16 + li;
      const uint32_t jc = (uint32_t)(col < nbc ? col : nbc - 1);
      Out o[MTMAX];
#pragma unroll
      for (int u = 0; u < MTMAX; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q) o[u][q] = 0;
      for (int s = 0; s < ks; ++s) {
        uint32_t off[M::KPL];
#pragma unroll
        for (int t = 0; t < M::KPL; ++t) {
          const int kk = s * M::KSTEP + gq * M::KPL + t;
          // padded K: a source row of the class (A is zero there; the row is
          // one this row gathers, so a non-finite value in it already makes
          // the row NaN)
          off[t] = so2[i0 + (kk < nx ? kk : 0)];
        }
        const Frag bf = M::load_b(cv, off, jc);
#pragma unroll
        for (int u = 0; u < MTMAX; ++u)
          if (u < mt) o[u] = M::mma(M::load_a(&At[(u * 16 + li) * lda + s * M::KSTEP + gq * M::KPL]), bf, o[u]);
      }
      if (col < nbc) {
#pragma unroll
        for (int u = 0; u < MTMAX; ++u) {
          if (u < mt) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int row = u * 16 + M::orow(gq, q);
              if (row < np_) {
                const uint32_t cd = pairS[(int64_t)plist[p0 + row] * nsb + col0 + col];
                if (cd != kInvalid) {
                  const double v = (double)o[u][q];
                  scatter_add<FIX>(&acc[cd >> 1], (cd & 1u) ? -v : v);
                }
              }
            }
          }
        }
      }
    }
    __syncthreads();  // the next class rebuilds the A tile
  }
  T *__restrict__ row = out + vo + g.off[a] + r * nc;
  for (int64_t j = tid; j < nc; j += 64 * NW) row[j] += row_value<FIX, T>(acc, j, finv, fbad);
}

size_t opp_mma_lds_bytes(int sA, int kstep, int pad, size_t asize, int npair, int64_t maxcol) {
  const int lda = (sA + kstep - 1) / kstep * kstep + pad;
  size_t b = (((size_t)maxcol * 8 + 15) & ~(size_t)15);
  b += (((size_t)kSymMmaRows * lda * asize) + 15) & ~(size_t)15;
  b += (((size_t)sA * 16 + 36) + 15) & ~(size_t)15;
  b += (size_t)sA * 8 + (size_t)npair * 4 + (size_t)sA * 4;
  return b;
}

size_t opp_pair_lds_bytes(int sA, size_t tsize, int npair, int64_t maxcol, int maxp8) {
  size_t b = (((size_t)maxcol * 8 + 15) & ~(size_t)15);
  size_t o1 = ((size_t)sA * 20 + 72 + 15) & ~(size_t)15;
  size_t o2 = (o1 + (size_t)sA * tsize + 7) & ~(size_t)7;
  size_t ow = (o2 + (size_t)sA * 8 + 15) & ~(size_t)15;
  return b + ow + (size_t)sA * maxp8 * tsize + (size_t)npair * 4;
}

// Beta pair codes re-addressed for the blocks: row kl, column = irrep-sorted
// index of the source string, code = (rank of the target in its irrep << 1) | sign.
__global__ void k_sym_pairs(const uint32_t *__restrict__ pair, int64_t ns_pad, int64_t nsb, int npair,
                            const int32_t *__restrict__ irr, const int32_t *__restrict__ pos,
                            const int64_t *__restrict__ start, uint32_t *__restrict__ out) {
  const int64_t J = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int kl = blockIdx.y;
  if (J >= nsb || kl >= npair) return;
  const uint32_t cd = pair[(int64_t)kl * ns_pad + J];
  const uint32_t nc = cd == kInvalid ? kInvalid : (((uint32_t)pos[cd >> 1]) << 1) | (cd & 1u);
  out[(int64_t)kl * nsb + start[irr[J]] + pos[J]] = nc;
}

size_t opp_lds_bytes(int sA, size_t tsize) {
  return (((size_t)sA * 20 + 36 + 15) & ~(size_t)15) + (size_t)sA * tsize;
}

// The pair form (row of sigma and the integral rows in LDS) up to this size:
// CAS(14,14) takes 53 KB in FP64, CAS(16,16) 93 KB.
constexpr size_t kSymPairLdsMax = kSymLdsCap;

SymArgs make_args(const SymInfo &S) {
  SymArgs g{};
  for (int a = 0; a < 9; ++a) {
    g.off[a] = S.off[a];
    g.startA[a] = S.startA[a];
  }
  for (int a = 0; a < 8; ++a) {
    g.rowsA[a] = S.cntA[a];
    g.ncol[a] = S.cntB[a ^ S.irrep];
    g.startBc[a] = S.startB[a ^ S.irrep];
  }
  return g;
}

// Irreps, ranks inside the irrep and the irrep-sorted index of one spin's
// strings, from the masks (host).
void spin_layout(const std::vector<uint64_t> &str, const int *orbsym, int norb,
                 std::vector<int32_t> &irr, std::vector<int32_t> &pos, std::vector<int32_t> &idx,
                 int64_t cnt[8], int64_t start[9]) {
  const int64_t ns = (int64_t)str.size();
  irr.resize(ns);
  pos.resize(ns);
  idx.resize(ns);
  for (int a = 0; a < 8; ++a) cnt[a] = 0;
  for (int64_t i = 0; i < ns; ++i) {
    int x = 0;
    for (int p = 0; p < norb; ++p)
      if ((str[i] >> p) & 1ull) x ^= orbsym[p];
    irr[i] = x;
    pos[i] = (int32_t)cnt[x]++;
  }
  start[0] = 0;
  for (int a = 0; a < 8; ++a) start[a + 1] = start[a] + cnt[a];
  for (int64_t i = 0; i < ns; ++i) idx[start[irr[i]] + pos[i]] = (int32_t)i;
}

template <typename T>
int upload(T **dst, const std::vector<T> &v, hipStream_t st) {
  SBCI_HIP(hipMalloc(dst, sizeof(T) * std::max<size_t>(v.size(), 1)));
  if (!v.empty())
    SBCI_HIP(hipMemcpyAsync(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, st));
  return SBCI_OK;
}

// Compacted same-spin lists of one spin (see k_sym_compact).
int compact_lists(sbci_ctx *ctx, const SpinTables &T, const int32_t *irr, const int32_t *pos,
                  const int64_t *start, int transposed, int *nfs, int32_t **col, double **v64,
                  float **v32) {
  const int64_t ns = T.ns;
  int32_t *cnt = nullptr;
  SBCI_HIP(hipMalloc(&cnt, sizeof(int32_t) * ns));
  const unsigned nb = (unsigned)((ns + 255) / 256);
  k_sym_count<<<nb, 256, 0, ctx->stream>>>(T.fcol, T.nf, ns, irr, cnt);
  SBCI_CHECK_LAUNCH();
  std::vector<int32_t> h(ns);
  SBCI_HIP(hipMemcpyAsync(h.data(), cnt, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, ctx->stream));
  SBCI_HIP(hipStreamSynchronize(ctx->stream));
  hipFree(cnt);
  int m = 1;
  for (int64_t i = 0; i < ns; ++i) m = std::max(m, (int)h[i]);
  *nfs = m;
  SBCI_HIP(hipMalloc(col, sizeof(int32_t) * ns * m));
  SBCI_HIP(hipMalloc(v64, sizeof(double) * ns * m));
  SBCI_HIP(hipMalloc(v32, sizeof(float) * ns * m));
  k_sym_compact<<<nb, 256, 0, ctx->stream>>>(T.fcol, T.fval64, T.nf, ns, irr, pos, m, start,
                                             transposed, *col, *v64, *v32);
  SBCI_CHECK_LAUNCH();
  return SBCI_OK;
}

}  // namespace

int setup_symmetry(sbci_ctx *ctx, const int *orbsym, int irrep, const double *h1,
                   const double *eri) {
  const int n = ctx->norb;
  if (irrep < 0 || irrep > 7) return set_error(SBCI_EINVAL, "irrep must be in [0, 7]");
  for (int p = 0; p < n; ++p)
    if (orbsym[p] < 0 || orbsym[p] > 7) return set_error(SBCI_EINVAL, "orbsym entries must be in [0, 7]");
  // totally symmetric integrals: the entries that break the symmetry must be
  // (numerically) zero, since the blocked sigma leaves them out
  double hmax = 0, gmax = 0;
  for (int i = 0; i < n * n; ++i) hmax = std::fmax(hmax, std::fabs(h1[i]));
  const size_t n4 = (size_t)n * n * n * n;
  for (size_t i = 0; i < n4; ++i) gmax = std::fmax(gmax, std::fabs(eri[i]));
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q)
      if (orbsym[p] != orbsym[q] && std::fabs(h1[p * n + q]) > 1e-10 * std::fmax(hmax, 1.0))
        return set_error(SBCI_EINVAL, "h1 couples orbitals of different irreps");
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q)
      for (int r = 0; r < n; ++r)
        for (int s = 0; s < n; ++s)
          if ((orbsym[p] ^ orbsym[q] ^ orbsym[r] ^ orbsym[s]) != 0 &&
              std::fabs(eri[(((size_t)p * n + q) * n + r) * n + s]) > 1e-10 * std::fmax(gmax, 1.0))
            return set_error(SBCI_EINVAL, "eri is not totally symmetric under orbsym");
  SymInfo *S = new SymInfo();
  ctx->sym = S;
  S->irrep = irrep;
  for (int p = 0; p < n; ++p) S->orbsym[p] = orbsym[p];
  hipStream_t st = ctx->stream;
  std::vector<uint64_t> sa(ctx->A.ns), sb(ctx->B.ns);
  SBCI_HIP(hipMemcpyAsync(sa.data(), ctx->A.str, sizeof(uint64_t) * ctx->A.ns, hipMemcpyDeviceToHost, st));
  SBCI_HIP(hipMemcpyAsync(sb.data(), ctx->B.str, sizeof(uint64_t) * ctx->B.ns, hipMemcpyDeviceToHost, st));
  SBCI_HIP(hipStreamSynchronize(st));
  std::vector<int32_t> irA, poA, ixA, irB, poB, ixB;
  spin_layout(sa, orbsym, n, irA, poA, ixA, S->cntA, S->startA);
  spin_layout(sb, orbsym, n, irB, poB, ixB, S->cntB, S->startB);
  S->off[0] = 0;
  for (int a = 0; a < 8; ++a) S->off[a + 1] = S->off[a] + S->cntA[a] * S->cntB[a ^ irrep];
  if (S->off[8] == 0) return set_error(SBCI_EINVAL, "no determinant has the requested irrep");
  if (S->off[8] >= ((int64_t)1 << 40)) return set_error(SBCI_EINVAL, "blocked space too large");
  SBCI_TRY(upload(&S->irrA, irA, st));
  SBCI_TRY(upload(&S->posA, poA, st));
  SBCI_TRY(upload(&S->idxA, ixA, st));
  SBCI_TRY(upload(&S->irrB, irB, st));
  SBCI_TRY(upload(&S->posB, poB, st));
  SBCI_TRY(upload(&S->idxB, ixB, st));
  std::vector<int32_t> os(orbsym, orbsym + n);
  SBCI_TRY(upload(&S->orbsym_d, os, st));
  std::vector<int64_t> sa9(S->startA, S->startA + 9), sb9(S->startB, S->startB + 9);
  int64_t *sad = nullptr, *sbd = nullptr;
  SBCI_TRY(upload(&sad, sa9, st));
  {
    const int rc = compact_lists(ctx, ctx->A, S->irrA, S->posA, sad, 0, &S->nfA, &S->colA,
                                 &S->valA64, &S->valA32);
    SBCI_HIP(hipStreamSynchronize(st));
    hipFree(sad);
    if (rc != SBCI_OK) return rc;
  }
  SBCI_TRY(upload(&sbd, sb9, st));
  {
    const int rc = compact_lists(ctx, ctx->B, S->irrB, S->posB, sbd, 1, &S->nfB, &S->colBT,
                                 &S->valBT64, &S->valBT32);
    if (rc != SBCI_OK) {
      hipFree(sbd);
      return rc;
    }
  }
  // pair form of the opposite-spin part: re-addressed beta pair codes and the
  // orbital pairs sorted by class
  {
    const int np = ctx->npair;
    std::vector<int32_t> pl;
    for (int x = 0; x < 8; ++x) {
      S->pcs[x] = (int)pl.size();
      for (int kk = 0, kl = 0; kk < n; ++kk)
        for (int l = 0; l <= kk; ++l, ++kl)
          if ((orbsym[kk] ^ orbsym[l]) == x) pl.push_back(kl);
    }
    S->pcs[8] = (int)pl.size();
    SBCI_TRY(upload(&S->plist, pl, st));
    const int64_t nsb = ctx->B.ns;
    SBCI_HIP(hipMalloc(&S->pairS, sizeof(uint32_t) * (size_t)np * nsb));
    k_sym_pairs<<<dim3((unsigned)((nsb + 255) / 256), (unsigned)np), 256, 0, st>>>(
        ctx->B.pair, ctx->B.ns_pad, nsb, np, S->irrB, S->posB, sbd, S->pairS);
    SBCI_CHECK_LAUNCH();
    SBCI_HIP(hipStreamSynchronize(st));
    hipFree(sbd);
    for (int a = 0; a < 8; ++a) S->maxcol = std::max<int64_t>(S->maxcol, S->cntB[a]);
  }
  // the diagonal in the blocked layout replaces the full-space one
  const SymArgs g = make_args(*S);
  const int64_t nd = S->off[8];
  double *d64 = nullptr;
  float *d32 = nullptr;
  SBCI_HIP(hipMalloc(&d64, sizeof(double) * nd));
  SBCI_HIP(hipMalloc(&d32, sizeof(float) * nd));
  const unsigned blocks = (unsigned)std::min<int64_t>((nd + 255) / 256, 8192);
  k_sym_gather<double><<<blocks, 256, 0, st>>>(g, S->idxA, S->idxB, ctx->B.ns, ctx->hdiag, d64);
  k_sym_gather<float><<<blocks, 256, 0, st>>>(g, S->idxA, S->idxB, ctx->B.ns, ctx->hdiag32, d32);
  SBCI_CHECK_LAUNCH();
  SBCI_HIP(hipStreamSynchronize(st));
  hipFree(ctx->hdiag);
  hipFree(ctx->hdiag32);
  ctx->hdiag = d64;
  ctx->hdiag32 = d32;
  ctx->ndet = nd;
  return SBCI_OK;
}

void free_symmetry(sbci_ctx *ctx) {
  SymInfo *S = ctx->sym;
  if (!S) return;
  hipFree(S->irrA);
  hipFree(S->posA);
  hipFree(S->idxA);
  hipFree(S->irrB);
  hipFree(S->posB);
  hipFree(S->idxB);
  hipFree(S->orbsym_d);
  hipFree(S->colA);
  hipFree(S->valA64);
  hipFree(S->valA32);
  hipFree(S->pairS);
  hipFree(S->plist);
  hipFree(S->colBT);
  hipFree(S->valBT64);
  hipFree(S->valBT32);
  delete S;
  ctx->sym = nullptr;
}

namespace {
template <typename M, typename T, bool FIX>
int launch_sym_mma(sbci_ctx *ctx, const SymArgs &g, const PairStarts &pcs, const T *W, size_t lds,
                   dim3 grid, const T *c, T *out, const double *rowmax) {
  const SymInfo &S = *ctx->sym;
  static bool attr = false;
  if (!attr) {
    SBCI_HIP(hipFuncSetAttribute((const void *)k_sym_opp_mma<M, T, FIX>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSymLdsCap));
    attr = true;
  }
  k_sym_opp_mma<M, T, FIX><<<grid, 256, lds, ctx->stream>>>(
      g, pcs, S.orbsym_d, S.idxA, S.posA, ctx->A.tab, ctx->A.s, S.pairS, ctx->B.ns, S.plist, W,
      ctx->npair, S.maxcol, c, out, rowmax, ctx->opp_wbound);
  return SBCI_OK;
}

template <typename T, bool FIX>
int launch_sym_pair(sbci_ctx *ctx, const SymArgs &g, const PairStarts &pcs, const T *W, size_t lds,
                    dim3 grid, int maxp8, const T *c, T *out, const double *rowmax) {
  const SymInfo &S = *ctx->sym;
  static bool attr = false;
  if (!attr) {
    SBCI_HIP(hipFuncSetAttribute((const void *)k_sym_opp_pair<T, FIX>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSymLdsCap));
    attr = true;
  }
  k_sym_opp_pair<T, FIX><<<grid, 256, lds, ctx->stream>>>(
      g, pcs, S.orbsym_d, S.idxA, S.posA, ctx->A.tab, ctx->A.s, S.pairS, ctx->B.ns, S.plist, W,
      ctx->npair, S.maxcol, maxp8, c, out, rowmax, ctx->opp_wbound);
  return SBCI_OK;
}

// bf16: the opposite-spin part on BF16 MFMA (T = float; the other parts in FP32)
template <typename T>
int sigma_sym_t(sbci_ctx *ctx, const T *c, T *out, int nvec, hipEvent_t *ev, bool bf16) {
  const SymInfo &S = *ctx->sym;
  const SymArgs g = make_args(S);
  const int64_t nd = S.off[8];
  constexpr bool dbl = std::is_same<T, double>::value;
  if (ev) SBCI_HIP(hipEventRecord(ev[0], ctx->stream));
  // beta part: rows staged in LDS in groups of kSymSameLdsRows when a group
  // of the longest rows fits in a third of a CU's LDS (three workgroups per
  // CU), otherwise gathered from global memory
  const size_t lds_same = (size_t)kSymSameLdsRows * (size_t)S.maxcol * sizeof(T);
  if (S.maxcol > 0 && lds_same <= kSymSameLdsMax) {
    RowGroups rl{};
    for (int a = 0; a < 8; ++a)
      rl.off[a + 1] = rl.off[a] + (g.ncol[a] > 0 ? (g.rowsA[a] + kSymSameLdsRows - 1) / kSymSameLdsRows : 0);
    if (rl.off[8] >= ((int64_t)1 << 31)) return set_error(SBCI_EINVAL, "blocked space too large");
    if (rl.off[8] > 0) {
      if constexpr (dbl)
        k_sym_same_lds<double, double, kSymSameLdsRows>
            <<<dim3((unsigned)rl.off[8], (unsigned)nvec), 256, lds_same, ctx->stream>>>(
                g, rl, S.colBT, S.valBT64, S.nfB, ctx->B.ns, c, out);
      else
        k_sym_same_lds<float, float, kSymSameLdsRows>
            <<<dim3((unsigned)rl.off[8], (unsigned)nvec), 256, lds_same, ctx->stream>>>(
                g, rl, S.colBT, S.valBT32, S.nfB, ctx->B.ns, c, out);
    }
  } else {
  RowGroups rg{};
  for (int a = 0; a < 8; ++a)
    rg.off[a + 1] = rg.off[a] + (g.rowsA[a] + kSymSameRows - 1) / kSymSameRows * g.ncol[a];
  const int64_t nblk = (rg.off[8] + 255) / 256;
  if (nblk >= ((int64_t)1 << 31)) return set_error(SBCI_EINVAL, "blocked space too large");
  if (nblk > 0) {
    if constexpr (dbl)
      k_sym_same<double, double><<<dim3((unsigned)nblk, (unsigned)nvec), 256, 0, ctx->stream>>>(
          g, rg, S.colBT, S.valBT64, S.nfB, ctx->B.ns, c, out);
    else
      k_sym_same<float, float><<<dim3((unsigned)nblk, (unsigned)nvec), 256, 0, ctx->stream>>>(
          g, rg, S.colBT, S.valBT32, S.nfB, ctx->B.ns, c, out);
  }
  }
  SBCI_CHECK_LAUNCH();
  // alpha same-spin part, block by block (rows of irrep a, lists in sorted order)
  for (int v = 0; v < nvec; ++v)
    for (int a = 0; a < 8; ++a) {
      const int64_t R = S.cntA[a], C = g.ncol[a];
      if (R == 0 || C == 0) continue;
      const int64_t lo = S.startA[a] * S.nfA;
      const void *vals;
      if constexpr (dbl) vals = S.valA64 + lo; else vals = S.valA32 + lo;
      SBCI_TRY(same_lists_block(ctx, S.colA + lo, vals, S.nfA, R, C, c + (int64_t)v * nd + S.off[a],
                                out + (int64_t)v * nd + S.off[a], dbl ? SBCI_F64 : SBCI_F32));
    }
  if (ev) SBCI_HIP(hipEventRecord(ev[1], ctx->stream));
  const SpinTables &A = ctx->A, &B = ctx->B;
  if (A.s > 0 && B.s > 0) {
    const T *W;
    if constexpr (dbl) W = ctx->W64; else W = ctx->W32;
    int maxp8 = 8, maxp = 0;
    for (int x = 0; x < 8; ++x) {
      maxp8 = std::max(maxp8, (S.pcs[x + 1] - S.pcs[x] + 7) & ~7);
      maxp = std::max(maxp, S.pcs[x + 1] - S.pcs[x]);
    }
    const size_t lp = opp_pair_lds_bytes(A.s, sizeof(T), ctx->npair, S.maxcol, maxp8);
    const dim3 grid((unsigned)A.ns, (unsigned)nvec);
    PairStarts pcs;
    for (int x = 0; x < 9; ++x) pcs.s[x] = S.pcs[x];
    // the MFMA form: classes of at most kSymMmaRows pairs, the block offsets
    // in 32 bits, its LDS within a CU's.  AUTO takes it for BF16 only: in
    // FP64 and FP32 the vector pair form below is faster at the measured
    // class sizes (CAS(14,14) irrep 0: 0.38 against 0.51 ms), the sums being
    // bound by the scatter, not the multiply-adds
    const int kstep = bf16 ? MBF16::KSTEP : dbl ? MF64::KSTEP : MF32::KSTEP;
    const int pad = bf16 ? MBF16::PAD : dbl ? MF64::PAD : MF32::PAD;
    const size_t asz = bf16 ? 2 : sizeof(T);
    const size_t lm = opp_mma_lds_bytes(A.s, kstep, pad, asz, ctx->npair, S.maxcol);
    const bool mma_ok = maxp <= kSymMmaRows && nd < ((int64_t)1 << 32) && lm <= kSymLdsCap;
    if (bf16 && !mma_ok)
      return set_error(SBCI_EINVAL, "blocked sigma: the BF16 form needs at most 64 pairs per class");
    if (bf16 && ctx->opp_form == SBCI_OPP_PAIR)
      return set_error(SBCI_EINVAL, "blocked sigma: the pair form has FP64 and FP32 flavours only");
    if (ctx->opp_form == SBCI_OPP_ORBITAL || ctx->opp_form == SBCI_OPP_ORBITAL_WINDOWED)
      return set_error(SBCI_EINVAL, "blocked sigma: the orbital form is not offered");
    if (ctx->opp_form == SBCI_OPP_CLASS_MFMA && !mma_ok)
      return set_error(SBCI_EINVAL, "blocked sigma: the MFMA form needs at most 64 pairs per class");
    const bool use_mma = bf16 || ctx->opp_form == SBCI_OPP_CLASS_MFMA;
    // FP64 in the pair and MFMA forms: each row's fixed-point scale needs
    // the largest |c| of every block row
    const bool fix = dbl && ctx->deterministic && (use_mma || lp <= kSymPairLdsMax);
    double *rmax = nullptr;
    if (fix) {
      SBCI_TRY(ensure(ctx->ws_rmax, sizeof(double) * (size_t)A.ns * nvec));
      rmax = static_cast<double *>(ctx->ws_rmax.ptr);
      k_sym_rowmax<<<grid, 256, 0, ctx->stream>>>(g, reinterpret_cast<const double *>(c), A.ns, rmax);
      SBCI_CHECK_LAUNCH();
    }
    if (use_mma) {
      if constexpr (dbl) {
        if (fix) SBCI_TRY((launch_sym_mma<MF64, double, true>(ctx, g, pcs, ctx->W64, lm, grid, c, out, rmax)));
        else SBCI_TRY((launch_sym_mma<MF64, double, false>(ctx, g, pcs, ctx->W64, lm, grid, c, out, rmax)));
      } else {
        if (bf16)
          SBCI_TRY((launch_sym_mma<MBF16, float, false>(ctx, g, pcs, ctx->W32, lm, grid, c, out, rmax)));
        else
          SBCI_TRY((launch_sym_mma<MF32, float, false>(ctx, g, pcs, ctx->W32, lm, grid, c, out, rmax)));
      }
    } else if (lp <= kSymPairLdsMax) {
      if (fix) SBCI_TRY((launch_sym_pair<T, true>(ctx, g, pcs, W, lp, grid, maxp8, c, out, rmax)));
      else SBCI_TRY((launch_sym_pair<T, false>(ctx, g, pcs, W, lp, grid, maxp8, c, out, rmax)));
    } else {
      const size_t lds = opp_lds_bytes(A.s, sizeof(T));
      if (lds > 64 * 1024) return set_error(SBCI_EINVAL, "blocked sigma: too many alpha excitations");
      k_sym_opp<T><<<grid, 256, lds, ctx->stream>>>(g, S.orbsym_d, S.idxA, S.idxB, S.posA, S.posB,
                                                    A.tab, A.s, B.tab, B.s, W, ctx->npair, c, out);
    }
    SBCI_CHECK_LAUNCH();
  }
  if (ev)
    for (int i = 2; i < 6; ++i) SBCI_HIP(hipEventRecord(ev[i], ctx->stream));
  return SBCI_OK;
}
}  // namespace

int sigma_sym(sbci_ctx *ctx, const void *c, void *out, int nvec, int mode, hipEvent_t *ev) {
  switch (mode) {
    case SBCI_F64:
      return sigma_sym_t<double>(ctx, static_cast<const double *>(c), static_cast<double *>(out),
                                 nvec, ev, false);
    case SBCI_F32:
      return sigma_sym_t<float>(ctx, static_cast<const float *>(c), static_cast<float *>(out),
                                nvec, ev, false);
    case SBCI_BF16:
      return sigma_sym_t<float>(ctx, static_cast<const float *>(c), static_cast<float *>(out),
                                nvec, ev, true);
    default:
      return set_error(SBCI_EINVAL, "unknown sigma dtype");
  }
}

int sym_blocks(const sbci_ctx *ctx, int64_t *out) {
  if (!ctx->sym) return set_error(SBCI_EINVAL, "context is not symmetry-blocked");
  const SymInfo &S = *ctx->sym;
  for (int a = 0; a < 8; ++a) {
    out[a] = S.cntA[a];
    out[8 + a] = S.cntB[a ^ S.irrep];
    out[16 + a] = S.off[a];
  }
  return SBCI_OK;
}

}  // namespace sbci
