// Internal declarations of libsbci: context layout, launch helpers, kernels'
// host-side launchers.  Not part of the public ABI (include/sbci.h).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sbci.h"

namespace sbci {

// 8-byte single-excitation record: E_pq |I> = sign |J>.
struct Ent {
  int32_t J;
  uint8_t p, q;
  int8_t sign;
  uint8_t pad;
};
static_assert(sizeof(Ent) == 8, "Ent must be 8 bytes");

// Scatter code of the pair tables: (target string << 1) | (sign < 0);
// kInvalid marks a pair that does not connect the string to any other.
constexpr uint32_t kInvalid = 0xffffffffu;
// Pair-table rows are padded with kInvalid (to 16 * (ceil(npair / 16) + 9)
// rows) so that the MFMA tiles of the opposite-spin kernel, in any grouping
// of at most 9 tiles, never need a row bound.

struct SpinTables {
  int m = 0;                // electrons of this spin
  int64_t ns = 0;           // number of strings C(norb, m)
  int s = 0;                // single excitations per string, m (norb - m + 1)
  int nf = 0;               // same-spin list length 1 + m(N-m) + C(m,2)C(N-m,2)
  uint64_t *str = nullptr;  // [ns]
  Ent *tab = nullptr;       // [ns][s]
  uint32_t *pair = nullptr; // [npair_pad][ns_pad] scatter codes
  int64_t ns_pad = 0;       // ns rounded up to 16 (pair-table row stride)
  // The pair table regrouped for the opposite-spin kernel: for 16-row tile u,
  // lane group g and column J, the four codes a lane scatters, in one 16-byte
  // load.  quad_r: rows u*16 + 4g + r (FP32 / BF16 MFMA output layout);
  // quad_s: rows u*16 + g + 4r (FP64 layout).  [npair_pad / 16][4][ns_pad].
  uint4 *quad_r = nullptr;
  uint4 *quad_s = nullptr;
  // Orbital-grouped scatter tables (the opposite-spin form for dilute
  // spaces): colq[q][j] is the j-th string (ascending) that holds orbital q,
  // nq = C(N-1, m-1) per orbital; qquad_r / qquad_s [q][mt][4][nq_pad] hold,
  // for 16-row tile u of orbitals p and lane group g, the scatter codes of
  // E_pq colq[q][j] for p = u*16 + 4g + r (qquad_r) or u*16 + g + 4r
  // (qquad_s), r = 0..3; columns j >= nq and orbitals p >= N are kInvalid.
  int64_t nq = 0, nq_pad = 0;
  int mt = 0;
  int32_t *colq = nullptr;
  uint4 *qquad_r = nullptr;
  uint4 *qquad_s = nullptr;
  int32_t *fcol = nullptr;  // [ns][nf] same-spin list columns
  double *fval64 = nullptr; // [ns][nf] FP64 values
  float *fval32 = nullptr;  // [ns][nf] FP32 values
  double *fdiag = nullptr;  // [ns] same-spin diagonal energy of each string
  // transposed lists [nf][ns], built when the LDS-staged same-spin kernel
  // applies (kSameLdsMinRows <= ns <= kSameLdsMaxRows)
  int32_t *fcolT = nullptr;
  double *fvalT64 = nullptr;
  float *fvalT32 = nullptr;
  // block-binned lists of the LDS-blocked same-spin kernel (ns above the
  // LDS-stripe range), built on first use: source rows in blocks of
  // kSameBlkRows; for 64-row group g and block b, slots boff[g*nblk + b] ..
  // boff[g*nblk + b + 1] - 1 hold one entry per row (lane) of the group:
  // bcol = column - b * kSameBlkRows (16 bits), values in FP64 and FP32;
  // rows with fewer entries in the block are padded with column 0, value 0.
  int nblk = 0;
  int64_t ngrp = 0;
  int32_t *boff = nullptr;     // [ngrp * nblk + 1]
  uint16_t *bcol = nullptr;    // [slots][64]
  double *bval64 = nullptr;    // [slots][64]
  float *bval32 = nullptr;     // [slots][64]
  // dense same-spin operator [ns][ns] (one-electron and same-spin parts),
  // built on first use by the dense form
  double *hd64 = nullptr;
  float *hd32 = nullptr;
  // BF16 form of the dense operator without its diagonal, and the diagonal
  // in FP32 (applied in the product's epilogue: it is too large to round)
  __hip_bfloat16 *hdbf = nullptr;
  float *hdd32 = nullptr;
  bool shared = false;      // aliases the alpha tables (n_alpha == n_beta)
};

// Row range of the LDS-staged same-spin kernel: a column stripe of 32 bytes
// per source row (8 FP32 or 4 FP64 columns) must fit in 120 KB of LDS, and
// below ~1024 rows the register-streaming kernel is already latency-bound.
constexpr int64_t kSameLdsMinRows = 1024;
constexpr int64_t kSameLdsMaxRows = 3840;
// LDS-blocked same-spin kernel above that range: source rows pass through
// LDS in blocks of kSameBlkRows rows x 64 bytes (8 FP64 or 16 FP32 columns;
// rows padded to 80 bytes, 160 KB); up to kSameBlkMaxBlocks blocks
// (block-local columns fit 16 bits).
constexpr int kSameBlkRows = 2048;
constexpr int kSameBlkMaxBlocks = 64;
// Dense same-spin form: chosen automatically above the LDS range when the
// lists hold at least a tenth of a row (there the MFMA product's extra flops
// cost less than streaming 8 bytes of source per list entry from L2); the
// dense operator takes ns^2 elements, so it is limited to 32768 strings.
constexpr int64_t kDenseMaxRows = 32768;

struct Workspace {
  void *ptr = nullptr;
  size_t bytes = 0;
};

struct Solver;  // SBCI1 driver state (solver.hip)

// Point-group blocking of a context (symmetry.hip): the determinants of one
// irrep, stored as blocks a = 0..7 of [alpha strings of irrep a] x [beta
// strings of irrep a ^ irrep], row-major, in order of a.
struct SymInfo {
  int irrep = 0;
  int orbsym[64] = {};
  int64_t cntA[8] = {}, cntB[8] = {};    // strings per irrep
  int64_t startA[9] = {}, startB[9] = {};// first irrep-sorted index per irrep
  int64_t off[9] = {};                   // block offsets; off[8] = blocked ndet
  int32_t *irrA = nullptr, *posA = nullptr, *idxA = nullptr;  // [nsa] irrep, rank in irrep, sorted -> global
  int32_t *irrB = nullptr, *posB = nullptr, *idxB = nullptr;  // [nsb]
  int32_t *orbsym_d = nullptr;           // [norb]
  // same-spin lists compacted to the string's own irrep (ranks and values):
  // alpha [irrep-sorted string][nfA], beta transposed [nfB][irrep-sorted string]
  int nfA = 0, nfB = 0;
  int32_t *colA = nullptr;
  double *valA64 = nullptr;
  float *valA32 = nullptr;
  int32_t *colBT = nullptr;
  double *valBT64 = nullptr;
  float *valBT32 = nullptr;
  // pair form of the opposite-spin part: beta pair codes with the target's
  // rank inside its irrep, columns in irrep-sorted order [npair][nsb], and
  // the orbital pairs sorted by class (orbsym[k] ^ orbsym[l]) with class starts
  uint32_t *pairS = nullptr;
  int32_t *plist = nullptr;
  int pcs[9] = {};
  int64_t maxcol = 0;                    // longest block row
};

}  // namespace sbci

struct sbci_ctx {
  int norb = 0, na = 0, nb = 0;
  int npair = 0;
  int npair_pad = 0;              // padded pair-table rows
  int64_t ndet = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t own_stream = nullptr;
  sbci::SpinTables A, B;
  int64_t *binom = nullptr;       // device [65][65]
  double *h1 = nullptr;           // device [N][N]
  double *eri = nullptr;          // device [N^4]
  double *W64 = nullptr;          // device [npair][npair] (kl|k'l')
  // s_beta * max_kl sum_k'l' |(kl|k'l')|: with max |C| over the rows an
  // output row gathers, a bound on every partial sum of the FP64
  // opposite-spin scatter (which accumulates in 64-bit fixed point)
  double opp_wbound = 0;
  bool deterministic = true;      // FP64 opposite-spin scatter in fixed point (sbci_set_deterministic)
  float *W32 = nullptr;
  __hip_bfloat16 *Wbf = nullptr;
  double *hdiag = nullptr;        // device [ndet]
  float *hdiag32 = nullptr;       // device [ndet]
  sbci::Workspace ws_t, ws_s;     // transposed input / output scratch of sigma
  sbci::Workspace ws_red;         // reduction partials + results
  sbci::Workspace ws_q;           // orbital-grouped copy of c (opposite-spin, dilute form)
  sbci::Workspace ws_rmax;        // max |C[J][.]| per alpha row and vector (FP64 opposite spin)
  int opp_form = 0;               // SBCI_OPP_AUTO / _PAIR / _ORBITAL
  int same_form = 0;              // SBCI_SAME_AUTO / _LISTS / _DENSE
  sbci::Solver *solver = nullptr;
  sbci::SymInfo *sym = nullptr;   // set when the context is symmetry-blocked
  bool trace_on = true;
  std::vector<sbci_step_info> trace;
  sbci_progress_fn progress = nullptr;
  void *progress_user = nullptr;
};

namespace sbci {

// ---- error handling (capi.hip) ----
int set_error(int code, const std::string &msg);
#define SBCI_HIP(call)                                                            \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      return ::sbci::set_error(e_ == hipErrorOutOfMemory ? SBCI_ENOMEM : SBCI_EDEVICE, \
                               std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)
#define SBCI_CHECK_LAUNCH()                                                       \
  do {                                                                            \
    hipError_t e_ = hipGetLastError();                                            \
    if (e_ != hipSuccess)                                                         \
      return ::sbci::set_error(SBCI_EDEVICE, std::string("kernel launch: ") +    \
                                                 hipGetErrorString(e_));          \
  } while (0)
#define SBCI_TRY(expr)          \
  do {                          \
    int r_ = (expr);            \
    if (r_ != SBCI_OK) return r_; \
  } while (0)

int ensure(Workspace &w, size_t bytes);

// ---- capi.hip ----
// Context on a given stream (own_stream = false leaves it to the caller);
// orbsym != NULL restricts it to the determinants of one irrep.
int create_context(int norb, int nalpha, int nbeta, const double *h1, const double *eri,
                   hipStream_t stream, bool own_stream, sbci_ctx **out,
                   const int *orbsym = nullptr, int irrep = 0);

// ---- symmetry.hip ----
// Block layout, compacted lists and the blocked diagonal; replaces ndet and
// hdiag by their blocked forms.
int setup_symmetry(sbci_ctx *ctx, const int *orbsym, int irrep, const double *h1,
                   const double *eri);
void free_symmetry(sbci_ctx *ctx);
// sigma on the blocked layout; ev (optional) receives 6 events around the
// same-spin part (ev[0..1]) and the opposite-spin part (ev[1..2]).
int sigma_sym(sbci_ctx *ctx, const void *c, void *out, int nvec, int mode, hipEvent_t *ev);
int sym_blocks(const sbci_ctx *ctx, int64_t *out);

// ---- tables.hip ----
int build_tables(sbci_ctx *ctx, const double *h1_host, const double *eri_host);
// block-binned same-spin lists of one spin (fields nblk .. bval32), from its
// row lists; allocates on the context stream
int build_blk_lists(sbci_ctx *ctx, SpinTables &T);
void free_tables(sbci_ctx *ctx);

// ---- sigma.hip ----
// sigma = H c for nvec vectors of element type T (double or float).
// mode: SBCI_F64 (T = double), SBCI_F32 or SBCI_BF16 (T = float).
int sigma(sbci_ctx *ctx, const void *c, void *out, int nvec, int mode);
// The same sigma with its scratch in a file-scope device array instead of
// allocated workspaces (no hipMalloc / hipFree): FP64 or FP32, list
// same-spin and pair opposite-spin forms, nvec * ndet * element size at most
// kNoAllocScratchBytes / 2; calls that overlap on one device race.
constexpr size_t kNoAllocScratchBytes = 64ull << 20;
constexpr int kMaxDevices = 64;
int sigma_noalloc(sbci_ctx *ctx, const void *c, void *out, int nvec, int mode);
// dst[r][q] += sum_e fval[r][e] src[fcol[r][e]][q] for one R x C matrix (one
// vector) with the L2-streaming list kernel; FP64 or FP32 (mode).
int same_lists_block(sbci_ctx *ctx, const int32_t *fcol, const void *fval, int nf, int64_t R,
                     int64_t C, const void *src, void *dst, int mode);
// Same, with HIP events around its five parts; ms[0..4] = alpha lists,
// opposite spin, transpose, beta lists, transposed add (milliseconds).
int sigma_profile(sbci_ctx *ctx, const void *c, void *out, int nvec, int mode, float *ms);
// opposite-spin form (SBCI_OPP_PAIR / SBCI_OPP_ORBITAL) used for this dtype
int opp_form(sbci_ctx *ctx, int mode, int *form);
// same-spin form (SBCI_SAME_LISTS / SBCI_SAME_DENSE) of one spin for a sigma dtype
int same_form(sbci_ctx *ctx, int spin, int dtype, int *form);

// ---- vec.hip: vector kernels with FP64 reductions ----
// Reductions write `nq` doubles to `out` (device); deterministic order.
template <typename T>
int dots(sbci_ctx *ctx, int64_t n, const T *a, const T *const *bs, int nb, double *out);
// b_i . b_j and b_i . h_j (i <= j) of a 4- or 6-vector FP64 basis in one pass
int gram(sbci_ctx *ctx, int64_t n, const double *const *b, const double *const *h, int m,
         double *out);
template <typename T>
int lincomb(sbci_ctx *ctx, int64_t n, T *out, const T *const *xs, const double *coef, int nx,
            double beta);
template <typename Td, typename Ts>
int convert(sbci_ctx *ctx, int64_t n, Td *dst, const Ts *src, double scale);

// Fused SBCI update pass (see vec.hip for the full contract).
struct UpdateArgs {
  double b, c, E, inv_norm, E0, floor, sx;
  int sy;          // 0: y_t treated as zero (segment start)
  int read_z;      // 0: z/Z not read (segment start, b = c = 0)
  int nconv;       // number of converged roots to project against (dots only)
  int want_zdots;  // 1: also reduce x.w, y.w, w.w (no deflation follows)
};
template <typename T>
int update(sbci_ctx *ctx, int64_t n, T *x, T *X, T *y, T *Y, const T *z, const T *Z, T *w,
           const T *D, const T *const *xc, const UpdateArgs &a, double *out);
template <typename T>
int deflate(sbci_ctx *ctx, int64_t n, T *w, const T *x, const T *y, const T *const *xc, int nconv,
            const double *d_coef, double *out);
template <typename T>
int dots_xyz(sbci_ctx *ctx, int64_t n, const T *x, const T *y, const T *z, const T *Z, double *out);
// Residual of one state: w = ((X - E x) * inv) / (D - E0) (|D - E0| floored),
// out[0] = |(X - E x) * inv|^2, out[1 + j] = xc_j . w.
template <typename T>
int resid(sbci_ctx *ctx, int64_t n, const T *x, const T *X, const T *D, double E, double inv,
          double E0, double floor, const T *const *xc, int nconv, T *w, double *out);

}  // namespace sbci
