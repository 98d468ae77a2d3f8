// Small dense eigenproblems of the SBCI step, shared by the host driver
// (solver.hip) and the device-resident batch solver (batch.hip).
//   jacobi_eigh  cyclic Jacobi, symmetric n x n (n <= NMAX), ascending
//   ritz_first   2x2 problem of a segment's first step (Eqs. S10-S24)
//   ritz_next    3x3 problem of later steps (Eqs. S33-S55)
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace sbci {

// Cyclic Jacobi for a symmetric n x n matrix (row-major, n <= NMAX),
// eigenvalues ascending in w, eigenvectors in the columns of V.
template <int NMAX>
__host__ __device__ inline void jacobi_eigh(int n, const double *Ain, double *w, double *V) {
  double A[NMAX * NMAX];
  for (int i = 0; i < n * n; ++i) A[i] = Ain[i];
  for (int i = 0; i < n * n; ++i) V[i] = 0;
  for (int i = 0; i < n; ++i) V[i * n + i] = 1;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0, tot = 0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += A[i * n + j] * A[i * n + j];
        if (i != j) off += A[i * n + j] * A[i * n + j];
      }
    if (off <= 1e-32 * tot || off == 0) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (apq == 0) continue;
        const double app = A[p * n + p], aqq = A[q * n + q];
        const double theta = (aqq - app) / (2 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1));
        const double c = 1 / sqrt(t * t + 1), s = t * c;
        for (int k = 0; k < n; ++k) {
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  // selection sort of the eigenpairs, ascending
  int idx[NMAX];
  for (int i = 0; i < n; ++i) idx[i] = i;
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j)
      if (A[idx[j] * n + idx[j]] < A[idx[i] * n + idx[i]]) {
        int t = idx[i];
        idx[i] = idx[j];
        idx[j] = t;
      }
  double Vs[NMAX * NMAX];
  for (int j = 0; j < n; ++j) {
    w[j] = A[idx[j] * n + idx[j]];
    for (int k = 0; k < n; ++k) Vs[k * n + j] = V[k * n + idx[j]];
  }
  for (int i = 0; i < n * n; ++i) V[i] = Vs[i];
}

// Result of the small Ritz problem: energies, coefficients of the lowest
// and second Ritz vectors on (x, y, z), and the update parameters.
struct Ritz {
  bool rank_ok = false, coef_ok = false;
  double E[3] = {0, 0, 0};
  double a1[3] = {0, 0, 0}, a2[3] = {0, 0, 0};
  double b = 0, c = 0, k = 0;
};

// First step of a segment: 2x2 problem in span{x, z} (Eqs. S10-S24).
__host__ __device__ inline Ritz ritz_first(double Nxx, double Nxz, double Nzz, double Hxx, double Hxz, double Hzz,
                double lindep) {
  Ritz r;
  const double Ax = 1.0 / sqrt(Nxx);            // x0 is normalised: Ax = 1 (Eq. S10)
  const double ux = Nxz * Ax;                        // xbar . z
  const double rad = Nzz - ux * ux;
  if (!(rad > lindep * fmax(Nzz, 1e-300))) return r;
  r.rank_ok = true;
  const double Bz = 1.0 / sqrt(rad);            // Eq. S12
  const double Bx = -ux * Bz * Ax;                   // Eq. S13 (zbar = Bz z + Bx x)
  const double V00 = Ax * Ax * Hxx;                  // Eq. S15a
  const double V01 = Ax * (Bx * Hxx + Bz * Hxz);     // Eq. S15b
  const double V11 = Bx * Bx * Hxx + Bz * Bz * Hzz + 2 * Bx * Bz * Hxz;  // Eq. S15c
  double Vm[4] = {V00, V01, V01, V11}, w[2], U[4];
  jacobi_eigh<2>(2, Vm, w, U);
  r.E[0] = w[0];
  r.E[1] = w[1];
  for (int i = 0; i < 2; ++i) {
    double vx = U[0 * 2 + i], vz = U[1 * 2 + i];
    double *a = i == 0 ? r.a1 : r.a2;
    a[0] = vx * Ax + vz * Bx;                        // Eq. S17
    a[1] = 0;
    a[2] = vz * Bz;
  }
  if (fabs(r.a1[0]) < lindep) return r;
  r.coef_ok = true;
  r.k = 1.0 / r.a1[0];                               // Eq. S23
  r.b = 1.0;
  r.c = -r.a1[2] / r.a1[0];                          // Eq. S24
  return r;
}

// Later step: 3x3 problem in span{x, y, z} (Eqs. S33-S55).
__host__ __device__ inline Ritz ritz_next(const double N[6], const double H[6], double lindep) {
  // N, H order: xx, xy, xz, yy, yz, zz
  Ritz r;
  const double Nxx = N[0], Nxy = N[1], Nxz = N[2], Nyy = N[3], Nyz = N[4], Nzz = N[5];
  const double Hxx = H[0], Hxy = H[1], Hxz = H[2], Hyy = H[3], Hyz = H[4], Hzz = H[5];
  const double Ax = 1.0 / sqrt(Nxx);                         // Eq. S34
  const double rady = Nyy - Nxy * Nxy / Nxx;
  if (!(rady > lindep * fmax(Nyy, 1e-300))) return r;
  const double By = 1.0 / sqrt(rady);                        // Eq. S36
  const double Bx = -(Nxy / Nxx) * By;                            // Eq. S37
  const double P = Bx * Nxz + By * Nyz;                           // Eq. S42
  const double radz = Nzz - Nxz * Nxz / Nxx - P * P;
  if (!(radz > lindep * fmax(Nzz, 1e-300))) return r;
  r.rank_ok = true;
  const double Cz = 1.0 / sqrt(radz);                        // Eq. S39
  const double Cy = -P * By * Cz;                                 // Eq. S40
  const double Cx = -(Nxz / Nxx + P * Bx) * Cz;                   // Eq. S41
  const double hxc = Cx * Hxx + Cy * Hxy + Cz * Hxz;              // x^T H zbar / 1
  const double hyc = Cx * Hxy + Cy * Hyy + Cz * Hyz;              // y^T H zbar
  double Vm[9];
  Vm[0] = Ax * Ax * Hxx;                                          // Eq. S44a
  Vm[1] = Vm[3] = Ax * (Bx * Hxx + By * Hxy);                     // Eq. S44b
  Vm[2] = Vm[6] = Ax * hxc;                                       // Eq. S44c
  Vm[4] = Bx * Bx * Hxx + By * By * Hyy + 2 * Bx * By * Hxy;      // Eq. S44d
  Vm[5] = Vm[7] = Bx * hxc + By * hyc;                            // Eq. S44e
  Vm[8] = Cx * Cx * Hxx + Cy * Cy * Hyy + Cz * Cz * Hzz + 2 * Cx * Cy * Hxy + 2 * Cx * Cz * Hxz +
          2 * Cy * Cz * Hyz;                                      // Eq. S44f
  double w[3], U[9];
  jacobi_eigh<3>(3, Vm, w, U);
  for (int i = 0; i < 3; ++i) r.E[i] = w[i];
  for (int i = 0; i < 2; ++i) {
    double vx = U[0 * 3 + i], vy = U[1 * 3 + i], vz = U[2 * 3 + i];
    double *a = i == 0 ? r.a1 : r.a2;
    a[0] = vx * Ax + vy * Bx + vz * Cx;                           // Eq. S46
    a[1] = vy * By + vz * Cy;
    a[2] = vz * Cz;
  }
  if (fabs(r.a1[0]) < lindep || fabs(r.a1[1]) < lindep) return r;
  r.coef_ok = true;
  r.k = 1.0 / r.a1[0];                                            // Eq. S53
  r.b = r.a1[1] / r.a1[0];                                        // Eq. S54
  r.c = -r.a1[2] / r.a1[1];                                       // Eq. S55
  return r;
}


}  // namespace sbci
