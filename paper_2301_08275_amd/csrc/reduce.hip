// Second-stage reductions and small pointwise kernels.
//
// Axis passes leave kRedSlots FP64 partial sums per workgroup.  One
// workgroup adds them in a fixed order (thread i takes partials i, i + 256,
// ... in turn, then a fixed tree), so the result does not depend on timing.
// For the imaginary-time method it also forms the renormalisation factor
// c = sqrt(norm_target / (dV sum |psi|^2)) on the device, so the step loop
// never waits on the host.
#include "gpe_kernels.h"

namespace gpe {
namespace {

constexpr int kFinThreads = 256;

__global__ void __launch_bounds__(kFinThreads)
finalize_kernel(const double *__restrict__ partial, long long count,
                double *__restrict__ out, double *__restrict__ scale_out,
                double norm_target, double dV, double shift_dt) {
  __shared__ double s[kRedSlots][kFinThreads];
  const int tid = threadIdx.x;
  double acc[kRedSlots];
#pragma unroll
  for (int k = 0; k < kRedSlots; ++k) acc[k] = 0;
  for (long long i = tid; i < count; i += kFinThreads) {
#pragma unroll
    for (int k = 0; k < kRedSlots; ++k) acc[k] += partial[i * kRedSlots + k];
  }
#pragma unroll
  for (int k = 0; k < kRedSlots; ++k) s[k][tid] = acc[k];
  __syncthreads();
  for (int h = kFinThreads / 2; h >= 1; h >>= 1) {
    if (tid < h) {
#pragma unroll
      for (int k = 0; k < kRedSlots; ++k) s[k][tid] += s[k][tid + h];
    }
    __syncthreads();
  }
  if (tid < kRedSlots) out[tid] = s[tid][0];
  if (tid == 0 && scale_out) {
    const double c = sqrt(norm_target / (dV * s[0][0]));
    scale_out[0] = c;
    if (shift_dt != 0.0) scale_out[1] += log(c) / shift_dt;
  }
}

// First stage of a two-stage finalize: workgroup b adds rows
// [b * chunk, min(count, (b + 1) * chunk)) in fixed order.
__global__ void __launch_bounds__(kFinThreads)
finalize_part_kernel(const double *__restrict__ partial, long long count, long long chunk,
                     double *__restrict__ out) {
  __shared__ double s[kRedSlots][kFinThreads];
  const int tid = threadIdx.x;
  const long long lo = (long long)blockIdx.x * chunk;
  const long long hi = lo + chunk < count ? lo + chunk : count;
  double acc[kRedSlots];
#pragma unroll
  for (int k = 0; k < kRedSlots; ++k) acc[k] = 0;
  for (long long i = lo + tid; i < hi; i += kFinThreads) {
#pragma unroll
    for (int k = 0; k < kRedSlots; ++k) acc[k] += partial[i * kRedSlots + k];
  }
#pragma unroll
  for (int k = 0; k < kRedSlots; ++k) s[k][tid] = acc[k];
  __syncthreads();
  for (int h = kFinThreads / 2; h >= 1; h >>= 1) {
    if (tid < h) {
#pragma unroll
      for (int k = 0; k < kRedSlots; ++k) s[k][tid] += s[k][tid + h];
    }
    __syncthreads();
  }
  if (tid < kRedSlots) out[(long long)blockIdx.x * kRedSlots + tid] = s[tid][0];
}

template <typename T>
__global__ void scale_kernel(T *__restrict__ psi, long long n, const double *__restrict__ c) {
  const double f = *c;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    psi[i] = (T)(f * (double)psi[i]);
}

__global__ void set_one_kernel(double *c) { *c = 1.0; }

// One workgroup per slot, after the last pass of step `step` of a chunk: the
// slots that ran that step form their renormalisation factor from their norm
// partials, in fixed order.
__global__ void __launch_bounds__(kFinThreads)
slot_update_kernel(Slot *__restrict__ slots, const double *__restrict__ partial,
                   long long blocks_per_grid, double dV, int step) {
  Slot &sl = slots[blockIdx.x];
  if (sl.mode != SLOT_IMAG || sl.steps_done + step >= sl.steps_total) return;
  __shared__ double s[kFinThreads];
  const int tid = threadIdx.x;
  const double *p = partial + (long long)blockIdx.x * blocks_per_grid * kRedSlots;
  double acc = 0;
  for (long long i = tid; i < blocks_per_grid; i += kFinThreads) acc += p[i * kRedSlots];
  s[tid] = acc;
  __syncthreads();
  for (int h = kFinThreads / 2; h >= 1; h >>= 1) {
    if (tid < h) s[tid] += s[tid + h];
    __syncthreads();
  }
  if (tid == 0) sl.scale = sqrt(sl.norm_target / (dV * s[0]));
}

__global__ void slot_advance_kernel(Slot *__restrict__ slots, int nslots, int steps) {
  for (int i = threadIdx.x; i < nslots; i += blockDim.x) {
    Slot &sl = slots[i];
    if (sl.mode == SLOT_FREE) continue;
    const int next = sl.steps_done + steps;
    sl.steps_done = next < sl.steps_total ? next : sl.steps_total;
  }
}

__global__ void slot_write_kernel(Slot *dst, Slot value) { *dst = value; }

__global__ void map_write_kernel(int *dst, SlotMap m) {
  for (int i = threadIdx.x; i < m.n; i += blockDim.x) dst[i] = m.idx[i];
}

template <typename S, typename D>
__global__ void convert_kernel(const S *__restrict__ src, D *__restrict__ dst, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = (D)src[i];
}

// Pseudo-random state for timing runs only (a hash of the index, values in
// [-1, 1)): data-dependent effects such as power draw then match a real run.
template <typename T>
__global__ void fill_noise_kernel(T *__restrict__ psi, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    unsigned long long z = (unsigned long long)i * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    psi[i] = (T)((double)(z >> 11) * 0x1.0p-52 - 1.0);
  }
}

unsigned grid_for(long long n, int threads) {
  long long b = (n + threads - 1) / threads;
  if (b > 65536) b = 65536;
  return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

hipError_t launch_finalize(const double *partial, long long count, double *out,
                           double *scale_out, double norm_target, double dV,
                           hipStream_t s, double *scratch, double shift_dt) {
  if (scratch && count > 4 * kFinThreads) {
    const long long chunk = (count + kFinBlocks - 1) / kFinBlocks;
    const int blocks = (int)((count + chunk - 1) / chunk);
    hipLaunchKernelGGL(finalize_part_kernel, dim3(blocks), dim3(kFinThreads), 0, s, partial,
                       count, chunk, scratch);
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kFinThreads), 0, s, scratch,
                       (long long)blocks, out, scale_out, norm_target, dV, shift_dt);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kFinThreads), 0, s, partial, count,
                     out, scale_out, norm_target, dV, shift_dt);
  return hipGetLastError();
}

hipError_t launch_slot_update(Slot *slots, int nslots, const double *partial,
                              long long blocks_per_grid, double dV, int step, hipStream_t s) {
  hipLaunchKernelGGL(slot_update_kernel, dim3(nslots), dim3(kFinThreads), 0, s, slots, partial,
                     blocks_per_grid, dV, step);
  return hipGetLastError();
}

hipError_t launch_slot_advance(Slot *slots, int nslots, int steps, hipStream_t s) {
  hipLaunchKernelGGL(slot_advance_kernel, dim3(1), dim3(256), 0, s, slots, nslots, steps);
  return hipGetLastError();
}

hipError_t launch_slot_write(Slot *dst, const Slot &value, hipStream_t s) {
  hipLaunchKernelGGL(slot_write_kernel, dim3(1), dim3(1), 0, s, dst, value);
  return hipGetLastError();
}

hipError_t launch_map_write(int *dst, const SlotMap &m, hipStream_t s) {
  if (m.n < 1 || m.n > kMaxSlots) return hipErrorInvalidValue;
  hipLaunchKernelGGL(map_write_kernel, dim3(1), dim3(256), 0, s, dst, m);
  return hipGetLastError();
}

hipError_t launch_scale(int precision, void *psi, long long sites, double *c,
                        hipStream_t s) {
  const long long n = 2 * sites;  // real components
  if (state_f32(precision))
    hipLaunchKernelGGL(scale_kernel<float>, dim3(grid_for(n, 256)), dim3(256), 0, s,
                       static_cast<float *>(psi), n, c);
  else
    hipLaunchKernelGGL(scale_kernel<double>, dim3(grid_for(n, 256)), dim3(256), 0, s,
                       static_cast<double *>(psi), n, c);
  hipLaunchKernelGGL(set_one_kernel, dim3(1), dim3(1), 0, s, c);
  return hipGetLastError();
}

hipError_t launch_fill_noise(int precision, void *psi, long long sites, hipStream_t s) {
  const long long n = 2 * sites;
  if (state_f32(precision))
    hipLaunchKernelGGL(fill_noise_kernel<float>, dim3(grid_for(n, 256)), dim3(256), 0, s,
                       static_cast<float *>(psi), n);
  else
    hipLaunchKernelGGL(fill_noise_kernel<double>, dim3(grid_for(n, 256)), dim3(256), 0, s,
                       static_cast<double *>(psi), n);
  return hipGetLastError();
}

hipError_t launch_convert(int src_prec, const void *src, int dst_prec, void *dst,
                          long long sites, hipStream_t s) {
  const long long n = 2 * sites;
  const dim3 g(grid_for(n, 256)), b(256);
  // storage types only: codes 1 and 2 both hold FP32 values
  src_prec = state_f32(src_prec) ? 1 : 0;
  dst_prec = state_f32(dst_prec) ? 1 : 0;
  if (src_prec == 0 && dst_prec == 1)
    hipLaunchKernelGGL((convert_kernel<double, float>), g, b, 0, s,
                       static_cast<const double *>(src), static_cast<float *>(dst), n);
  else if (src_prec == 1 && dst_prec == 0)
    hipLaunchKernelGGL((convert_kernel<float, double>), g, b, 0, s,
                       static_cast<const float *>(src), static_cast<double *>(dst), n);
  else if (src_prec == 1)
    hipLaunchKernelGGL((convert_kernel<float, float>), g, b, 0, s,
                       static_cast<const float *>(src), static_cast<float *>(dst), n);
  else
    hipLaunchKernelGGL((convert_kernel<double, double>), g, b, 0, s,
                       static_cast<const double *>(src), static_cast<double *>(dst), n);
  return hipGetLastError();
}

}  // namespace gpe
