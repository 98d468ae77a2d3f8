// Host-side sanitizer driver: every entry point of libsbci on small cases
// (the library's host code built with AddressSanitizer; GPU code unchanged).
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "sbci.h"
#include <sanitizer/lsan_interface.h>
#include <unistd.h>

#define CHECK(x) do { int rc_ = (x); if (rc_ != 0 && rc_ != SBCI_ENOCONV) { \
  std::printf("FAIL %s -> %d (%s)\n", #x, rc_, sbci_last_error()); std::exit(1); } } while (0)

static void integrals(int n, unsigned seed, const std::vector<int> *orbsym, std::vector<double> &h1,
                      std::vector<double> &eri) {
  unsigned s = seed * 2654435761u + 12345u;
  auto rnd = [&]() { s = s * 1664525u + 1013904223u; return ((s >> 8) & 0xffff) / 65536.0 - 0.5; };
  auto ok = [&](int p, int q) { return !orbsym || (*orbsym)[p] == (*orbsym)[q]; };
  h1.assign(n * n, 0.0);
  for (int p = 0; p < n; ++p)
    for (int q = 0; q <= p; ++q)
      if (ok(p, q)) h1[p * n + q] = h1[q * n + p] = (p == q ? -2.0 + 0.3 * p : 0.1 * rnd());
  const int K = 2 * n;
  std::vector<double> L(K * n * n, 0.0);
  for (int k = 0; k < K; ++k)
    for (int p = 0; p < n; ++p)
      for (int q = 0; q <= p; ++q)
        if (ok(p, q)) L[(k * n + p) * n + q] = L[(k * n + q) * n + p] = 0.3 * rnd() / (1 + k);
  eri.assign((size_t)n * n * n * n, 0.0);
  for (int k = 0; k < K; ++k)
    for (int pq = 0; pq < n * n; ++pq)
      for (int rs = 0; rs < n * n; ++rs) eri[(size_t)pq * n * n + rs] += L[k * n * n + pq] * L[k * n * n + rs];
}

static void run_ctx(sbci_ctx *ctx, int nroots) {
  const int64_t nd = sbci_ndet(ctx);
  double *c, *s, *vec;
  hipMalloc(&c, 8 * nd * 2);
  hipMalloc(&s, 8 * nd * 2);
  hipMalloc(&vec, 8 * nd * nroots);
  std::vector<double> hc(2 * nd);
  for (int64_t i = 0; i < 2 * nd; ++i) hc[i] = std::sin(0.37 * i + 1.0);
  hipMemcpy(c, hc.data(), 8 * 2 * nd, hipMemcpyHostToDevice);
  CHECK(sbci_hdiag(ctx, s));
  CHECK(sbci_sigma(ctx, c, s, 2, SBCI_F64));
  std::vector<float> hf(2 * nd);
  for (int64_t i = 0; i < 2 * nd; ++i) hf[i] = (float)hc[i];
  hipMemcpy(c, hf.data(), 4 * 2 * nd, hipMemcpyHostToDevice);
  CHECK(sbci_sigma(ctx, c, s, 2, SBCI_F32));
  CHECK(sbci_sigma(ctx, c, s, 1, SBCI_BF16));
  sbci_opts o;
  sbci_default_opts(&o);
  std::vector<double> e(nroots);
  sbci_report rep;
  for (int prec : {SBCI_F64, SBCI_F32, SBCI_BF16}) {
    o.precision = prec;
    CHECK(sbci_solve(ctx, nroots, 1e-10, &o, e.data(), vec, &rep));
  }
  o.precision = SBCI_F64;
  CHECK(sbci_davidson(ctx, nroots, 1e-10, &o, e.data(), vec, &rep));
  CHECK(sbci_solve2(ctx, nroots, 1e-10, &o, e.data(), vec, &rep));
  CHECK(sbci_begin(ctx, nroots, 1e-10, &o));
  int done = 0, guard = 0;
  sbci_step_info info;
  for (int k = 0; k < 2 && !done; ++k) CHECK(sbci_step(ctx, &info, &done));
  if (!done) CHECK(sbci_iterate(ctx, c));   // checkpoint of the running root
  while (!done && guard++ < 5000) CHECK(sbci_step(ctx, &info, &done));
  CHECK(sbci_finish(ctx, e.data(), vec, &rep));
  if (sbci_iterate(ctx, c) == 0) { std::printf("FAIL iterate after the last root\n"); std::exit(1); }
  if (nroots >= 2) {
    // resume after nroots - 1 converged roots, with and without their energies,
    // in FP64 and FP32 (host Gram-Schmidt and the root pools)
    std::vector<double> hv(nd * (nroots - 1));
    hipMemcpy(hv.data(), vec, 8 * nd * (nroots - 1), hipMemcpyDeviceToHost);
    std::vector<double> ek(e.begin(), e.end() - 1);
    o.nconv0 = nroots - 1;
    o.xc0 = hv.data();
    for (int prec : {SBCI_F64, SBCI_F32}) {
      o.precision = prec;
      o.ec0 = prec == SBCI_F64 ? ek.data() : nullptr;
      CHECK(sbci_solve(ctx, nroots, 1e-10, &o, e.data(), vec, &rep));
    }
    if (sbci_davidson(ctx, nroots, 1e-10, &o, e.data(), vec, &rep) == 0) { std::printf("FAIL resume refusal\n"); std::exit(1); }
    o.nconv0 = 0;
    o.xc0 = o.ec0 = nullptr;
    o.precision = SBCI_F64;
  }
  std::vector<sbci_step_info> tr(64);
  if (sbci_trace(ctx, tr.data(), 64) < 0) { std::printf("FAIL trace\n"); std::exit(1); }
  // refusals: bad dtype, aliasing, nroots out of range
  if (sbci_sigma(ctx, c, c, 1, SBCI_F64) == 0 || sbci_sigma(ctx, c, s, 1, 7) == 0 ||
      sbci_solve(ctx, 0, 1e-10, &o, e.data(), vec, &rep) == 0) { std::printf("FAIL refusal\n"); std::exit(1); }
  hipFree(c);
  hipFree(s);
  hipFree(vec);
}

int main() {
  setvbuf(stdout, nullptr, _IONBF, 0);
  std::vector<double> h1, eri;
  int cases[][4] = {{6, 3, 3, 2}, {7, 3, 4, 2}, {5, 0, 2, 1}, {8, 4, 4, 3}};
  for (auto &k : cases) {
    integrals(k[0], k[0] + k[1], nullptr, h1, eri);
    sbci_ctx *ctx = nullptr;
    CHECK(sbci_create(k[0], k[1], k[2], h1.data(), eri.data(), &ctx));
    run_ctx(ctx, k[3]);
    CHECK(sbci_destroy(ctx));
    std::printf("case %d %d %d ok\n", k[0], k[1], k[2]);
  }
  {
    std::vector<int> orb = {0, 1, 2, 3, 0, 1, 2, 3};
    integrals(8, 3, &orb, h1, eri);
    sbci_ctx *ctx = nullptr;
    CHECK(sbci_create_sym(8, 4, 4, h1.data(), eri.data(), orb.data(), 0, &ctx));
    run_ctx(ctx, 2);
    CHECK(sbci_destroy(ctx));
    std::printf("sym ok\n");
  }
  {
    const int ni = 6;
    std::vector<std::vector<double>> H(ni), E(ni);
    std::vector<const double *> hp(ni), ep(ni);
    int norb[ni], na[ni], nb[ni], nr[ni];
    for (int i = 0; i < ni; ++i) {
      norb[i] = 5 + i % 4; na[i] = nb[i] = norb[i] / 2; nr[i] = 1 + i % 3;
      integrals(norb[i], 100 + i, nullptr, H[i], E[i]);
      hp[i] = H[i].data(); ep[i] = E[i].data();
    }
    sbci_batch *b = nullptr;
    CHECK(sbci_batch_create(ni, norb, na, nb, hp.data(), ep.data(), &b));
    sbci_opts o;
    sbci_default_opts(&o);
    std::vector<double> e(3 * ni);
    std::vector<sbci_batch_inst> info(ni);
    sbci_batch_report rep;
    CHECK(sbci_batch_solve(b, nr, 1e-10, &o, nullptr, e.data(), info.data(), &rep));
    sbci_batch_config best, cand[16];
    double ms[16];
    int nc = 16;
    CHECK(sbci_batch_tune(b, nr, 1e-10, &o, &best, ms, cand, &nc));
    o.precision = SBCI_BF16;
    CHECK(sbci_batch_solve(b, nr, 1e-10, &o, &best, e.data(), info.data(), &rep));
    double *v;
    hipMalloc(&v, 8 * sbci_batch_ndet(b, 0) * 3);
    CHECK(sbci_batch_vectors(b, 0, v));
    hipFree(v);
    CHECK(sbci_batch_destroy(b));
    std::printf("batch ok\n");
  }
  // leak check now; then leave without the HIP runtime teardown, which the
  // sanitizer runtime does not survive
  __lsan_do_leak_check();
  std::printf("ALL_OK\n");
  _exit(0);
}
