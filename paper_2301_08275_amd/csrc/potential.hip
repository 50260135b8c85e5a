// Per-axis tables of a separable analytic potential (the anharmonic traps,
// optical lattices and time-dependent potentials V(r, t) of Eq. 2 that the
// paper's feature list names): V(r) = sum_j v_j(x_j) with
//   v_j(x) = hw_j (x - c_j)^2 + a_j (x - c_j)^4 + s_j sin^2(q_j x + phi_j).
// The fused passes read V at a site as three table entries (L1/L2 resident:
// at most 3 x 1024 doubles), so the potential costs no per-site HBM traffic.
// A table holds a weighted sum of v_j at two parameter sets, the mean of the
// potential over the two midpoints a fused N(dt) step covers.
#include "gpe_kernels.h"

namespace gpe {
namespace {

__device__ __forceinline__ double sep_value(const SepParams &P, int j, double x) {
  const double d = x - P.c[j], d2 = d * d;
  const double sn = sin(P.q[j] * x + P.ph[j]);
  return P.hw[j] * d2 + P.a[j] * d2 * d2 + P.s[j] * sn * sn;
}

__global__ void vtables_kernel(const SepParams A, double wA, const SepParams B, double wB,
                               int n0, int n1, int n2, double lo0, double lo1, double lo2,
                               double h0, double h1, double h2, double *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n0 + n1 + n2) return;
  const int j = i < n0 ? 0 : (i < n0 + n1 ? 1 : 2);
  const int k = i - (j == 0 ? 0 : (j == 1 ? n0 : n0 + n1));
  const double x = (j == 0 ? lo0 : j == 1 ? lo1 : lo2) + k * (j == 0 ? h0 : j == 1 ? h1 : h2);
  double v = wA * sep_value(A, j, x);
  if (wB != 0) v += wB * sep_value(B, j, x);
  out[i] = v;
}

}  // namespace

hipError_t launch_vtables(const SepParams &A, double wA, const SepParams &B, double wB,
                          const int n[3], const double lo[3], const double h[3], double *out,
                          hipStream_t s) {
  const int total = n[0] + n[1] + n[2];
  hipLaunchKernelGGL(vtables_kernel, dim3((total + 255) / 256), dim3(256), 0, s, A, wA, B, wB,
                     n[0], n[1], n[2], lo[0], lo[1], lo[2], h[0], h[1], h[2], out);
  return hipGetLastError();
}

}  // namespace gpe
