// |k|-shell spectra: particle number, compressible and incompressible kinetic
// energy, and the quantum-pressure part.  The particle-number kernel also
// sums |k|^2 |psi_hat|^2 over the grid: the kinetic energy by Parseval's
// identity on the whole grid.
//
// The spectra of Z_j = u_j + i w_j (two real fields packed in one complex FFT)
// are unpacked per wavenumber from Z_j(k) and Z_j(-k):
//   U_j(k) = (Z_j(k) + conj(Z_j(-k))) / 2,  W_j(k) = (Z_j(k) - conj(Z_j(-k))) / (2i),
// U is split into k (k.U)/|k|^2 (compressible) and the rest (incompressible;
// k = 0 belongs there), and |.|^2 is summed per shell round(|k|/dk).  Every
// sum is taken in a fixed order, so the spectra are bitwise reproducible: a
// wavefront adds the runs of equal shells among its lanes by a fixed-order
// scan and accumulates them, in its own program order, into a histogram of
// its own in LDS; the workgroup adds its wavefronts' histograms in wavefront
// order; a second kernel adds the workgroup histograms in workgroup order.
#include "gpe_kernels.h"

namespace gpe {
namespace {

constexpr int kShellThreads = 256;
constexpr int kShellU0 = 4, kShellU1 = 2;  // sites per thread per iteration (kind 0, 1)

template <typename T>
struct alignas(2 * sizeof(T)) cxs {
  T x, y;
};

// Signed mode of index i on an n-point axis (the Nyquist index n/2 is
// negative; an axis of one point, a missing axis of the 3D view, is mode 0).
__device__ __forceinline__ int mode_of(int i, int n) { return i < (n + 1) / 2 ? i : i - n; }

__device__ __forceinline__ int log2_of(int n) { return 31 - __clz(n); }

// Lane moves of the wavefront scan (DPP: register reads across lanes, no
// LDS): row_shr:d takes lane i - d within a row of 16 lanes, row_bcast:15
// gives lane 15 of each row to the next row (written into rows 1 and 3),
// row_bcast:31 gives lane 31 to rows 2 and 3.  A lane without a source (or
// outside the rows written) gets `old`.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_move(int v, int old) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)dpp_move<CTRL, ROWS>((int)b, 0);
  const int hi = dpp_move<CTRL, ROWS>((int)(b >> 32), 0);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | lo));
}

// One step of the segmented scan: add the moved partial sums whose key (the
// run they belong to) equals this lane's.  A lane with no source gets key -2,
// which no lane carries.
template <int NV, int CTRL, int ROWS>
__device__ __forceinline__ void scan_step(double (&x)[NV], int key) {
  const int ky = dpp_move<CTRL, ROWS>(key, -2);
  double y[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) y[v] = dpp_move<CTRL, ROWS>(x[v]);
  if (ky == key)
#pragma unroll
    for (int v = 0; v < NV; ++v) x[v] += y[v];
}

// Inclusive sums of x over the run of equal keys that ends at this lane (runs
// of a key are contiguous in lane order): a segmented scan, first within
// rows of 16 lanes (shifts by 1, 2, 4, 8), then across rows (lane 15 into
// the next row, lane 31 into the upper half).  After a step a lane holds the
// sum over its run within a window ending at the lane; since a run is
// contiguous, a partial sum with the same key belongs to the lane's run.
// Every lane must be active; the order of the additions is fixed.
template <int NV>
__device__ __forceinline__ void run_sums(double (&x)[NV], int key) {
  scan_step<NV, 0x111, 0xf>(x, key);
  scan_step<NV, 0x112, 0xf>(x, key);
  scan_step<NV, 0x114, 0xf>(x, key);
  scan_step<NV, 0x118, 0xf>(x, key);
  scan_step<NV, 0x142, 0xa>(x, key);
  scan_step<NV, 0x143, 0xc>(x, key);
}

// Site geometry: indices, wavevector, shell and run key (see shell_kernel).
struct ShellSite {
  long long s, ms;
  int i2, bin, key;
  bool on, pairs;
  double k[3], kk;
};

template <int KIND>
__device__ __forceinline__ ShellSite shell_site(const ShellArgs &a, long long s, bool valid,
                                                int l1, int l2) {
  const int n0 = a.n[0], n1 = a.n[1], n2 = a.n[2];
  ShellSite q;
  q.s = s;
  // (grids hold at most 2^30 sites: the index fits 32 bits)
  const unsigned su = (unsigned)s;
  q.i2 = (int)(su & (n2 - 1));
  const unsigned r = su >> l2;
  const int i1 = (int)(r & (n1 - 1)), i0 = (int)(r >> l1);
  // Kind 1: the decomposed energies at the mirror site (index -i) equal
  // those at i when the mirror's wavevector is -k (u and w are transforms
  // of real fields); that fails only on a Nyquist index (n/2 is its own
  // mirror with the same k) of a used axis.  Such pairs count once from the
  // half i2 <= n2/2, twice for 0 < i2 < n2/2; other sites count once (the
  // index ranges of kind 1 visit exactly these sites, see shell_range).
  q.pairs = (2 * i0 != n0 || a.kscale[0] == 0) && (2 * i1 != n1 || a.kscale[1] == 0);
  q.on = valid;
  const int m0 = mode_of(i0, n0), m1 = mode_of(i1, n1), m2 = mode_of(q.i2, n2);
  q.k[0] = a.kscale[0] * m0;
  q.k[1] = a.kscale[1] * m1;
  q.k[2] = a.kscale[2] * m2;
  q.kk = q.k[0] * q.k[0] + q.k[1] * q.k[1] + q.k[2] * q.k[2];
  int bin;
  if (a.integer_shells) {
    // shell t: (2t - 1)^2 <= 4 M < (2t + 1)^2, i.e. t = floor(sqrt(M) + 1/2),
    // settled in integers without branches (|m_j| <= 512, so M < 2^20 and
    // 4 M and the squares fit in 32 bits): r = floor(sqrt(M)) from an FP32
    // root (off by at most one; checked both ways), then t = r + 1 exactly
    // when 4 M > (2r + 1)^2 (they cannot be equal: one is even, one odd)
    const int M = m0 * m0 + m1 * m1 + m2 * m2;
    int r = (int)sqrtf((float)M);
    r -= r * r > M ? 1 : 0;
    r += (r + 1) * (r + 1) <= M ? 1 : 0;
    bin = r + ((2 * r + 1) * (2 * r + 1) < 4 * M ? 1 : 0);
  } else {
    bin = (int)floor(sqrt(q.kk) / a.dk + 0.5);
  }
  q.bin = bin < a.nbins ? bin : a.nbins - 1;  // the clamp is unreachable for the shell count used
  q.key = q.on ? (int)(((r & 0x3fff) << 13) | ((2 * q.i2 >= n2) ? 1 << 12 : 0) | q.bin) : -1;
  q.ms = (long long)(((((unsigned)((n0 - i0) & (n0 - 1)) * n1 + ((n1 - i1) & (n1 - 1))) << l2) |
                      ((n2 - q.i2) & (n2 - 1))));
  return q;
}

// Add v (the sum of a run of equal shells, held by the run's last lane) to
// bin `bin` of this wavefront's histogram h.  The 64 sites of a wavefront are
// consecutive and aligned: when the last axis has at least 128 points they
// lie in one half of one row, where the shell index is monotone, so the runs
// of one instruction have distinct bins and update h together; otherwise
// runs of different rows may share a bin and the last lanes add one at a
// time in lane order.
__device__ __forceinline__ void add_run(double *h, int bin, double v, bool last, bool rows_apart,
                                        int lane) {
  if (!rows_apart) {
    if (last) h[bin] += v;
    return;
  }
  unsigned long long m = __ballot(last);
  while (m) {
    const int l = __ffsll((unsigned long long)m) - 1;
    if (lane == l) h[bin] += v;
    m &= m - 1;
  }
}

// Index ranges of a shell launch.  Kind 0 visits every site (RANGE_ALL).
// Kind 1 counts each pair of wavevectors k, -k once: RANGE_HALF visits the
// lower half-row i2 < n2/2 of every row (index e: row e / (n2/2), i2 =
// e mod (n2/2)); RANGE_EXTRA then visits the column i2 = n2/2 of every row,
// and the upper half-row of each row with a Nyquist index on a used axis
// (such a row is its own mirror, so all of its sites count).
enum { RANGE_ALL = 0, RANGE_HALF = 1, RANGE_EXTRA = 2 };

// Rows with a Nyquist index on a used axis: i0 = n0/2 (n1 rows), then
// i1 = n1/2 (n0 rows, less the one already listed).
__device__ __forceinline__ long long nyquist_rows(const ShellArgs &a) {
  const bool u0 = a.kscale[0] != 0, u1 = a.kscale[1] != 0;
  return (u0 ? a.n[1] : 0) + (u1 ? a.n[0] : 0) - (u0 && u1 ? 1 : 0);
}

__device__ __forceinline__ long long range_count(const ShellArgs &a, int range) {
  const long long rows = (long long)a.n[0] * a.n[1];
  if (range == RANGE_ALL) return rows * a.n[2];
  if (range == RANGE_HALF) return rows * (a.n[2] / 2);
  return rows + nyquist_rows(a) * (a.n[2] / 2 - 1);
}

template <int RANGE>
__device__ __forceinline__ long long site_of(const ShellArgs &a, long long e, int l2) {
  if constexpr (RANGE == RANGE_ALL) {
    return e;
  } else if constexpr (RANGE == RANGE_HALF) {
    const int h2 = l2 - 1;
    return ((e >> h2) << l2) | (e & ((1LL << h2) - 1));
  } else {
    const int n0 = a.n[0], n1 = a.n[1], n2 = a.n[2];
    const long long rows = (long long)n0 * n1;
    if (e < rows) return (e << l2) | (n2 / 2);
    e -= rows;
    const long long per = n2 / 2 - 1;
    const long long r = e / per;
    const int t = (int)(e - r * per);
    const bool u0 = a.kscale[0] != 0;
    int i0, i1;
    if (u0 && r < n1) {
      i0 = n0 / 2;
      i1 = (int)r;
    } else {
      const int r2 = (int)(r - (u0 ? n1 : 0));
      i1 = n1 / 2;
      i0 = (u0 && r2 >= n0 / 2) ? r2 + 1 : r2;
    }
    return (((long long)i0 * n1 + i1) << l2) | (n2 / 2 + 1 + t);
  }
}

// Every lane of a wavefront runs the same number of iterations (the shuffles
// need them all); a lane past the end of the range carries key -1.  Within a
// wavefront the sites are consecutive indices of the range: for RANGE_ALL
// and RANGE_HALF, within one row (fixed i0, i1) and one half of the last
// axis the shell index is monotone in i2, so equal bins form contiguous runs
// keyed by (row, half, bin); each run is summed across lanes in fixed order
// and added to the wavefront's histogram by its last lane.  The few sites of
// RANGE_EXTRA lie in different rows, and their last lanes add one at a time.
// Each iteration takes U blocks of sites and issues all their loads before
// any arithmetic.
template <typename T, int KIND, int U, int RANGE>
__device__ __forceinline__ void shell_range(const ShellArgs &a, double *h, bool rows_apart,
                                            int l1, int l2, int lane, double &kin) {
  constexpr int NF = KIND == 0 ? 1 : 3;
  const int nb = a.nbins, n2 = a.n[2];
  const long long count = range_count(a, RANGE);
  const cxs<T> *fs[3] = {static_cast<const cxs<T> *>(a.f[0]),
                         static_cast<const cxs<T> *>(a.f[1]),
                         static_cast<const cxs<T> *>(a.f[2])};
  const long long step = (long long)gridDim.x * blockDim.x * U;
  for (long long e0 = (long long)blockIdx.x * blockDim.x * U; e0 < count; e0 += step) {
    ShellSite q[U];
    cxs<T> zp[U][NF], zm[U][NF];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long e = e0 + (long long)u * blockDim.x + threadIdx.x;
      const bool valid = e < count;
      q[u] = shell_site<KIND>(a, valid ? site_of<RANGE>(a, e, l2) : 0, valid, l1, l2);
    }
    // Every lane loads (a lane with nothing to add reads element 0) and the
    // values are zeroed afterwards: loads under per-lane branches end up in
    // blocks of their own, each waiting for its data before the next load
    // issues.
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      if (fs[j]) {  // (uniform: a missing axis has no field)
#pragma unroll
        for (int u = 0; u < U; ++u) {
          zp[u][j] = fs[j][q[u].on ? q[u].s : 0];
          zm[u][j] = KIND != 0 ? fs[j][q[u].on ? q[u].ms : 0] : cxs<T>{0, 0};
        }
      } else {
#pragma unroll
        for (int u = 0; u < U; ++u) zp[u][j] = zm[u][j] = cxs<T>{0, 0};
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int j = 0; j < NF; ++j)
        if (!q[u].on) zp[u][j] = zm[u][j] = cxs<T>{0, 0};
    // kind 0: the weighted |Z|^2 of each site, formed once all loads are
    // issued, and this thread's running |k|^2 |Z|^2 sum (in program order)
    double en[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double z2 = (double)zp[u][0].x * zp[u][0].x + (double)zp[u][0].y * zp[u][0].y;
      en[u] = a.w * z2;
      if constexpr (KIND == 0) kin += a.wk * q[u].kk * z2;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int key_next = __shfl_down(q[u].key, 1, 64);
      const bool last = q[u].on && (lane == 63 || key_next != q[u].key);
      if constexpr (KIND == 0) {
        double e[1] = {en[u]};
        run_sums(e, q[u].key);
        add_run(h, q[u].bin, e[0], last, rows_apart, lane);
      } else {
        double csum = 0, isum = 0, qsum = 0;
        if (q[u].on) {
          const int i2 = q[u].i2;
          const double wgt = (q[u].pairs && i2 != 0 && 2 * i2 != n2) ? a.w : 0.5 * a.w;
          double ur[3], ui[3];
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            ur[j] = 0.5 * ((double)zp[u][j].x + (double)zm[u][j].x);
            ui[j] = 0.5 * ((double)zp[u][j].y - (double)zm[u][j].y);
            const double wr = 0.5 * ((double)zp[u][j].y + (double)zm[u][j].y);
            const double wi = -0.5 * ((double)zp[u][j].x - (double)zm[u][j].x);
            qsum += wr * wr + wi * wi;
          }
          const double *kv = q[u].k, kk = q[u].kk;
          if (kk > 0) {
            const double ikk = 1.0 / kk;  // one division per site
            const double pr = (kv[0] * ur[0] + kv[1] * ur[1] + kv[2] * ur[2]) * ikk;
            const double pi = (kv[0] * ui[0] + kv[1] * ui[1] + kv[2] * ui[2]) * ikk;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
              const double cr = kv[j] * pr, ci = kv[j] * pi;
              csum += cr * cr + ci * ci;
              isum += (ur[j] - cr) * (ur[j] - cr) + (ui[j] - ci) * (ui[j] - ci);
            }
          } else {
#pragma unroll
            for (int j = 0; j < 3; ++j) isum += ur[j] * ur[j] + ui[j] * ui[j];
          }
          csum *= wgt;
          isum *= wgt;
          qsum *= wgt;
        }
        double sums[3] = {csum, isum, qsum};
        run_sums(sums, q[u].key);
        add_run(h, q[u].bin, sums[0], last, rows_apart, lane);
        add_run(h + nb, q[u].bin, sums[1], last, rows_apart, lane);
        add_run(h + 2 * nb, q[u].bin, sums[2], last, rows_apart, lane);
      }
    }
  }
}

template <typename T, int KIND, int U>
__global__ void __launch_bounds__(kShellThreads) shell_kernel(const ShellArgs a) {
  // one histogram (kind 0: particle number) or three (kind 1: compressible,
  // incompressible, quantum pressure) of nbins per wavefront
  constexpr int NH = KIND == 0 ? 1 : 3;
  extern __shared__ double hist[];
  const int nb = a.nbins, nw = blockDim.x >> 6;
  for (int i = threadIdx.x; i < nw * NH * nb; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  double *h = hist + (threadIdx.x >> 6) * NH * nb;
  const int l1 = log2_of(a.n[1]), l2 = log2_of(a.n[2]);
  const int lane = threadIdx.x & 63;
  double kin = 0;
  if constexpr (KIND == 0) {
    shell_range<T, 0, U, RANGE_ALL>(a, h, a.n[2] < 128, l1, l2, lane, kin);
  } else {
    // a wavefront's 64 half-row indices share one half-row when n2/2 >= 64
    shell_range<T, 1, U, RANGE_HALF>(a, h, a.n[2] < 128, l1, l2, lane, kin);
    shell_range<T, 1, 1, RANGE_EXTRA>(a, h, true, l1, l2, lane, kin);
  }
  // kind 0: the workgroup's |k|^2 sum, lanes by a fixed butterfly (lane 0's
  // result), then the wavefronts in order
  __shared__ double kin_wave[kShellThreads / 64];
  if constexpr (KIND == 0) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) kin += __shfl_xor(kin, o, 64);
    if (lane == 0) kin_wave[threadIdx.x >> 6] = kin;
  }
  __syncthreads();
  // row of this workgroup: kind 0 N(n) in [0, nb) and the |k|^2 sum at nb;
  // kind 1 the energies in [nb, 4 nb)
  double *out = a.partial + (long long)blockIdx.x * 4 * nb;
  for (int i = threadIdx.x; i < 4 * nb; i += blockDim.x) {
    const int j = KIND == 0 ? i : i - nb;  // index within the wavefront histograms
    double t = 0;
    if (j >= 0 && j < NH * nb) {
      for (int w = 0; w < nw; ++w) t += hist[w * NH * nb + j];
    } else if (KIND == 0 && i == nb) {
      for (int w = 0; w < nw; ++w) t += kin_wave[w];
    }
    out[i] = t;
  }
}

// Column sums of a [count][len] array in fixed order: a block of 64 columns
// x 16 row groups; group g adds rows g, g + 16, ... in order, then the 16
// group sums are added in order.
constexpr int kSumCols = 64, kSumGroups = 16;

__global__ void __launch_bounds__(kSumCols * kSumGroups)
sum_columns_kernel(const double *__restrict__ partial, long long count, int len,
                   double *__restrict__ out) {
  __shared__ double part[kSumGroups][kSumCols];
  const int c = threadIdx.x % kSumCols, g = threadIdx.x / kSumCols;
  const int i = blockIdx.x * kSumCols + c;
  double s = 0;
  if (i < len)
    for (long long b = g; b < count; b += kSumGroups) s += partial[b * len + i];
  part[g][c] = s;
  __syncthreads();
  if (g == 0 && i < len) {
    double t = part[0][c];
    for (int k = 1; k < kSumGroups; ++k) t += part[k][c];
    out[i] = t;
  }
}

// Workgroup shape of a shell launch: as many wavefronts (at most four) as
// have room for their histograms in 64 KiB of LDS.
struct ShellShape {
  int waves;
  size_t lds;
};
ShellShape shell_shape(int kind, int nbins) {
  const size_t per_wave = (kind == 0 ? 1 : 3) * (size_t)nbins * sizeof(double);
  int waves = (int)((64 * 1024) / per_wave);
  if (waves > kShellThreads / 64) waves = kShellThreads / 64;
  return {waves, waves > 0 ? waves * per_wave : 0};
}

const void *shell_fn(int precision, int kind) {
  // the packed fields are stored like the state
  if (state_f32(precision))
    return kind == 0 ? (const void *)shell_kernel<float, 0, kShellU0>
                     : (const void *)shell_kernel<float, 1, kShellU1>;
  return kind == 0 ? (const void *)shell_kernel<double, 0, kShellU0>
                   : (const void *)shell_kernel<double, 1, kShellU1>;
}

}  // namespace

// Every workgroup loops over an equal share of the sites, so the launch is
// one round of the workgroups the device holds at once (a second, partial
// round would leave most CUs idle), capped by the sites and kShellMaxBlocks.
// The count depends only on the device and the grid: the fixed-order sums
// stay bitwise reproducible.
int shell_blocks(int precision, int kind, long long sites, int nbins) {
  const ShellShape sh = shell_shape(kind, nbins);
  if (sh.waves < 1) return 1;
  long long b = (sites + 64LL * sh.waves - 1) / (64LL * sh.waves);
  if (b > kShellMaxBlocks) b = kShellMaxBlocks;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, shell_fn(precision, kind),
                                                   64 * sh.waves, sh.lds) == hipSuccess &&
      cus > 0 && per_cu > 0 && (long long)cus * per_cu < b)
    b = (long long)cus * per_cu;
  return (int)(b < 1 ? 1 : b);
}

hipError_t launch_shells(int precision, const ShellArgs &a, int blocks, hipStream_t s) {
  const ShellShape sh = shell_shape(a.kind, a.nbins);
  if (sh.waves < 1 || blocks < 1 || blocks > kShellMaxBlocks) return hipErrorInvalidValue;
  const dim3 threads(64 * sh.waves);
  if (state_f32(precision)) {
    if (a.kind == 0)
      hipLaunchKernelGGL((shell_kernel<float, 0, kShellU0>), dim3(blocks), threads, sh.lds, s, a);
    else
      hipLaunchKernelGGL((shell_kernel<float, 1, kShellU1>), dim3(blocks), threads, sh.lds, s, a);
  } else {
    if (a.kind == 0)
      hipLaunchKernelGGL((shell_kernel<double, 0, kShellU0>), dim3(blocks), threads, sh.lds, s, a);
    else
      hipLaunchKernelGGL((shell_kernel<double, 1, kShellU1>), dim3(blocks), threads, sh.lds, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_sum_columns(const double *partial, long long count, int len, double *out,
                              hipStream_t s) {
  hipLaunchKernelGGL(sum_columns_kernel, dim3((len + kSumCols - 1) / kSumCols),
                     dim3(kSumCols * kSumGroups), 0, s, partial, count, len, out);
  return hipGetLastError();
}

}  // namespace gpe
