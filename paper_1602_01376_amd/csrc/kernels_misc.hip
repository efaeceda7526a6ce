// Small element-wise kernels: reduced-system assembly (eq. (11),
// written row-major as the batched LU expects),
// precision conversions and the FP64 vector steps of iterative refinement.
#include "device_util.hpp"
#include "internal.hpp"

namespace invaskit {
namespace {

template <typename TZ, typename TV>
__global__ __launch_bounds__(256) void k_zform(const ZformProb* __restrict__ probs) {
  const ZformProb p = probs[blockIdx.x];
  const int n = p.sr + p.sl;
  const gptr<TZ> Z = glb(static_cast<TZ*>(p.Z));
  const gptr<const TV> pr = glb(static_cast<const TV*>(p.pr));
  const gptr<const TV> pl = glb(static_cast<const TV*>(p.pl));
  for (int64_t idx = threadIdx.x; idx < (int64_t)n * n; idx += 256) {
    const int i = (int)(idx / n), j = (int)(idx % n);  // row-major
    TZ v;
    if (i < p.sr) {
      v = (j < p.sr) ? TZ(i == j) : (TZ)pr[(int64_t)(j - p.sr) * p.sr + i];
    } else {
      v = (j < p.sr) ? (TZ)pl[(int64_t)j * p.sl + (i - p.sr)] : TZ(i == j);
    }
    Z[idx] = v;
  }
}

// dst = src + shift * I for one square block of order m (either storage
// order: the diagonal is every (m+1)-th element), one workgroup per block
template <typename T>
__global__ __launch_bounds__(256) void k_copy_shift(const CopyShiftProb* __restrict__ probs) {
  const CopyShiftProb p = probs[blockIdx.x];
  const gptr<const T> src = glb(static_cast<const T*>(p.src));
  const gptr<T> dst = glb(static_cast<T*>(p.dst));
  const int64_t mm = (int64_t)p.m * p.m;
  const T sh = (T)p.shift;
  for (int64_t e = threadIdx.x; e < mm; e += 256)
    dst[e] = src[e] + ((e % (p.m + 1)) == 0 ? sh : T(0));
}

__global__ void k_convert(const double* __restrict__ in, float* __restrict__ out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}

template <typename TI, typename TO>
__global__ void k_copy_cols(const TI* __restrict__ in, int64_t ldi, TO* __restrict__ out,
                            int64_t ldo, int64_t n, const double* __restrict__ scale, int inv) {
  const int c = blockIdx.y;
  double s = 1.0;
  if (scale) s = inv ? (scale[c] > 0 ? 1.0 / scale[c] : 0.0) : scale[c];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[c * ldo + i] = (TO)((double)in[c * ldi + i] * s);
}

__global__ void k_sqrt_cols(const double* __restrict__ norm2, double* __restrict__ scale,
                            int ncols) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < ncols) scale[c] = sqrt(norm2[c]);
}

template <typename TD>
__global__ void k_axpy_cols(double* __restrict__ x, int64_t ldx, const TD* __restrict__ d,
                            int64_t ldd, int64_t n, const double* __restrict__ scale) {
  const int c = blockIdx.y;
  const double s = scale[c];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[c * ldx + i] += s * (double)d[c * ldd + i];
}

// Multi-dot, first pass: the rows of column c are cut into nblk chunks;
// block (b, c, k) sums V_k[i, c] * w[i, c] over chunk b and writes
// part[(k * ncols + c) * nblk + b].  V_k = V + k * vstride, column c at
// + c * ldv.  The four waves' sums are added in a fixed order, so the result
// does not depend on scheduling.
__global__ __launch_bounds__(256) void k_dots_part(const double* __restrict__ V, int64_t vstride,
                                                   int64_t ldv, const double* __restrict__ w,
                                                   int64_t ldw, int64_t n, int64_t chunk,
                                                   double* __restrict__ part) {
  __shared__ double wsum[4];
  const int b = blockIdx.x, c = blockIdx.y, k = blockIdx.z;
  const int nblk = gridDim.x, ncols = gridDim.y;
  const double* __restrict__ v = V + k * vstride + c * ldv;
  const double* __restrict__ x = w + c * ldw;
  const int64_t i1 = min(n, (int64_t)(b + 1) * chunk);
  double acc = 0.0;
  for (int64_t i = (int64_t)b * chunk + threadIdx.x; i < i1; i += 256) acc = fma(v[i], x[i], acc);
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0)
    part[((int64_t)k * ncols + c) * nblk + b] = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
}

// Multi-dot, second pass: out[t] = sum over b of part[t * nblk + b], one
// workgroup per output (nblk <= 256): one partial per thread, summed by the
// same butterfly in every wave and the four waves in a fixed order.
__global__ __launch_bounds__(256) void k_dots_sum(const double* __restrict__ part, int nblk,
                                                  double* __restrict__ out) {
  __shared__ double wsum[4];
  const int t = blockIdx.x;
  double v = (int)threadIdx.x < nblk ? part[(int64_t)t * nblk + threadIdx.x] : 0.0;
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) out[t] = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
}

// out[i, c] += alpha * sum_k coef[k * ncols + c] * V_k[i, c]
__global__ void k_lincomb(double* __restrict__ out, int64_t ldo, const double* __restrict__ V,
                          int64_t vstride, int64_t ldv, int nk, const double* __restrict__ coef,
                          double alpha, int64_t n) {
  const int c = blockIdx.y, ncols = gridDim.y;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int k = 0; k < nk; ++k) acc = fma(coef[k * ncols + c], V[k * vstride + c * ldv + i], acc);
    out[c * ldo + i] += alpha * acc;
  }
}

// v[i, c] *= scale[c], in place
__global__ void k_scale_cols(double* __restrict__ v, int64_t ld, int64_t n,
                             const double* __restrict__ scale) {
  const int c = blockIdx.y;
  const double s = scale[c];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    v[c * ld + i] *= s;
}

// v[i, c] = 0
__global__ void k_zero_cols(double* __restrict__ v, int64_t ld, int64_t n) {
  const int c = blockIdx.y;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    v[c * ld + i] = 0.0;
}

int grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

template <typename TZ, typename TV>
hipError_t launch_zform(const ZformProb* probs, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_zform<TZ, TV>), dim3(count), dim3(256), 0, s, probs);
  return hipGetLastError();
}
template hipError_t launch_zform<double, double>(const ZformProb*, int, hipStream_t);
template hipError_t launch_zform<float, float>(const ZformProb*, int, hipStream_t);
template hipError_t launch_zform<double, float>(const ZformProb*, int, hipStream_t);

template <typename T>
hipError_t launch_copy_shift(const CopyShiftProb* probs, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_copy_shift<T>), dim3(count), dim3(256), 0, s, probs);
  return hipGetLastError();
}
template hipError_t launch_copy_shift<double>(const CopyShiftProb*, int, hipStream_t);
template hipError_t launch_copy_shift<float>(const CopyShiftProb*, int, hipStream_t);

hipError_t launch_convert_f64_f32(const double* in, float* out, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_convert, dim3(grid_for(n)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

template <typename TI, typename TO>
hipError_t launch_copy_cols(const TI* in, int64_t ldi, TO* out, int64_t ldo, int64_t n,
                            int ncols, const double* scale, bool invert_scale, hipStream_t s) {
  if (n <= 0 || ncols <= 0) return hipSuccess;
  const int g = (grid_for(n) + ncols - 1) / ncols + 1;
  hipLaunchKernelGGL((k_copy_cols<TI, TO>), dim3(g, ncols), dim3(256), 0, s, in, ldi, out, ldo, n,
                     scale, invert_scale ? 1 : 0);
  return hipGetLastError();
}
template hipError_t launch_copy_cols<double, double>(const double*, int64_t, double*, int64_t,
                                                     int64_t, int, const double*, bool,
                                                     hipStream_t);
template hipError_t launch_copy_cols<double, float>(const double*, int64_t, float*, int64_t,
                                                    int64_t, int, const double*, bool,
                                                    hipStream_t);
template hipError_t launch_copy_cols<float, double>(const float*, int64_t, double*, int64_t,
                                                    int64_t, int, const double*, bool,
                                                    hipStream_t);

hipError_t launch_sqrt_cols(const double* norm2, double* scale, int ncols, hipStream_t s) {
  if (ncols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sqrt_cols, dim3((ncols + 255) / 256), dim3(256), 0, s, norm2, scale, ncols);
  return hipGetLastError();
}

template <typename TD>
hipError_t launch_axpy_cols(double* x, int64_t ldx, const TD* d, int64_t ldd, int64_t n,
                            int ncols, const double* scale, hipStream_t s) {
  if (n <= 0 || ncols <= 0) return hipSuccess;
  const int g = (grid_for(n) + ncols - 1) / ncols + 1;
  hipLaunchKernelGGL(k_axpy_cols<TD>, dim3(g, ncols), dim3(256), 0, s, x, ldx, d, ldd, n, scale);
  return hipGetLastError();
}
template hipError_t launch_axpy_cols<float>(double*, int64_t, const float*, int64_t, int64_t, int,
                                            const double*, hipStream_t);
template hipError_t launch_axpy_cols<double>(double*, int64_t, const double*, int64_t, int64_t,
                                             int, const double*, hipStream_t);

int dots_blocks(int64_t n) {
  int64_t nb = (n + 4095) / 4096;
  if (nb > 256) nb = 256;
  if (nb < 1) nb = 1;
  return (int)nb;
}

size_t dots_part_doubles(int64_t n, int nk, int ncols) {
  return (size_t)dots_blocks(n) * nk * ncols;
}

hipError_t launch_dots(const double* V, int64_t vstride, int64_t ldv, int nk, const double* w,
                       int64_t ldw, int64_t n, int ncols, double* part, double* out,
                       hipStream_t s) {
  if (nk <= 0 || ncols <= 0) return hipSuccess;
  const int nblk = dots_blocks(n);
  const int64_t chunk = (n + nblk - 1) / nblk;
  hipLaunchKernelGGL(k_dots_part, dim3(nblk, ncols, nk), dim3(256), 0, s, V, vstride, ldv, w,
                     ldw, n, chunk, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dots_sum, dim3(nk * ncols), dim3(256), 0, s, part, nblk, out);
  return hipGetLastError();
}

hipError_t launch_lincomb(double* out, int64_t ldo, const double* V, int64_t vstride,
                          int64_t ldv, int nk, const double* coef, int ncols, double alpha,
                          int64_t n, hipStream_t s) {
  if (nk <= 0 || ncols <= 0 || n <= 0) return hipSuccess;
  const int g = (grid_for(n) + ncols - 1) / ncols + 1;
  hipLaunchKernelGGL(k_lincomb, dim3(g, ncols), dim3(256), 0, s, out, ldo, V, vstride, ldv, nk,
                     coef, alpha, n);
  return hipGetLastError();
}

hipError_t launch_scale_cols(double* v, int64_t ld, int64_t n, int ncols, const double* scale,
                             hipStream_t s) {
  if (n <= 0 || ncols <= 0) return hipSuccess;
  const int g = (grid_for(n) + ncols - 1) / ncols + 1;
  hipLaunchKernelGGL(k_scale_cols, dim3(g, ncols), dim3(256), 0, s, v, ld, n, scale);
  return hipGetLastError();
}

hipError_t launch_zero_cols(double* v, int64_t ld, int64_t n, int ncols, hipStream_t s) {
  if (n <= 0 || ncols <= 0) return hipSuccess;
  const int g = (grid_for(n) + ncols - 1) / ncols + 1;
  hipLaunchKernelGGL(k_zero_cols, dim3(g, ncols), dim3(256), 0, s, v, ld, n);
  return hipGetLastError();
}

}  // namespace invaskit
