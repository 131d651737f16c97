// Fourier-mode MLP surrogate of the collision operator (not part of the paper): BF16
// MFMA GEMMs with FP32 accumulation for training and inference, fused bias/SiLU
// epilogues, MSE loss, Adam, the low-mode feature extraction from the spectral path's
// fhat, and the moment-residual indicator with fallback compaction.
//
// GEMM: C[M x N] = A[M x K] . B[K x N] on v_mfma_f32_32x32x16_bf16.  Operand layouts:
// A is "MK" (row-major, K contiguous) or "KM" (K rows, M contiguous); B is "NK" (each of
// the N columns stored K-contiguous, i.e. weights [out][in]) or "KN".  Tiles of 128 x 128
// x 32 are staged through LDS K-contiguous, so one kernel serves the forward product
// (A=MK, B=NK), the input gradient (A=MK, B=KN) and the weight gradient (A=KM, B=KN).
// M, N, K must be multiples of 128, 128 and 32.
#include <hip/hip_runtime.h>

#include "fks_internal.hpp"

namespace fks {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int GBM = 128, GBN = 128, GBK = 32, GPAD = 8, GLD = GBK + GPAD;  // LDS row stride (bf16)

__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu_f(float z) {
  const float s = 1.0f / (1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// Epilogues
enum GemmEpi {
  kEpiF32 = 0,        // Cf = acc (+ bias)
  kEpiBiasSilu = 1,   // Cf = z = acc + bias (pre-activation, kept for backward), Ch = bf16(silu(z))
  kEpiDSilu = 2,      // Ch = bf16(acc * silu'(Zin))
  kEpiBiasBf16 = 3    // Ch = bf16(acc + bias)
};

template <bool A_KM, bool B_KN, int EPI>
__global__ __launch_bounds__(256) void k_gemm(const __bf16* __restrict__ A, const __bf16* __restrict__ B, int M,
                                              int N, int K, int lda, int ldb, const float* __restrict__ bias,
                                              float* __restrict__ Cf, __bf16* __restrict__ Ch,
                                              const float* __restrict__ Zin, int ldc) {
  __shared__ __align__(16) __bf16 As[GBM * GLD];
  __shared__ __align__(16) __bf16 Bs[GBN * GLD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * GBM, n0 = blockIdx.x * GBN;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  f32x16 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;

  for (int k0 = 0; k0 < K; k0 += GBK) {
    // ---- stage A tile (GBM x GBK) as As[m][k]
    if constexpr (!A_KM) {
      const int r = tid >> 1, kh = (tid & 1) * 16;
      const uint4* src = reinterpret_cast<const uint4*>(A + size_t(m0 + r) * lda + k0 + kh);
      uint4* dst = reinterpret_cast<uint4*>(As + r * GLD + kh);
      dst[0] = src[0];
      dst[1] = src[1];
    } else {
      const int kr = tid >> 3, mc = (tid & 7) * 16;
      const uint4* src = reinterpret_cast<const uint4*>(A + size_t(k0 + kr) * lda + m0 + mc);
      uint4 v0 = src[0], v1 = src[1];
      const __bf16* h0 = reinterpret_cast<const __bf16*>(&v0);
      const __bf16* h1 = reinterpret_cast<const __bf16*>(&v1);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        As[(mc + i) * GLD + kr] = h0[i];
        As[(mc + 8 + i) * GLD + kr] = h1[i];
      }
    }
    // ---- stage B tile (GBK x GBN) as Bs[n][k]
    if constexpr (!B_KN) {
      const int r = tid >> 1, kh = (tid & 1) * 16;
      const uint4* src = reinterpret_cast<const uint4*>(B + size_t(n0 + r) * ldb + k0 + kh);
      uint4* dst = reinterpret_cast<uint4*>(Bs + r * GLD + kh);
      dst[0] = src[0];
      dst[1] = src[1];
    } else {
      const int kr = tid >> 3, nc = (tid & 7) * 16;
      const uint4* src = reinterpret_cast<const uint4*>(B + size_t(k0 + kr) * ldb + n0 + nc);
      uint4 v0 = src[0], v1 = src[1];
      const __bf16* h0 = reinterpret_cast<const __bf16*>(&v0);
      const __bf16* h1 = reinterpret_cast<const __bf16*>(&v1);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        Bs[(nc + i) * GLD + kr] = h0[i];
        Bs[(nc + 8 + i) * GLD + kr] = h1[i];
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GBK; kk += 16) {
      bf16x8 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a[i] = *reinterpret_cast<const bf16x8*>(As + (wm + i * 32 + (lane & 31)) * GLD + kk + 8 * (lane >> 5));
        b[i] = *reinterpret_cast<const bf16x8*>(Bs + (wn + i * 32 + (lane & 31)) * GLD + kk + 8 * (lane >> 5));
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // ---- epilogue: lane holds rows 8*(e/4) + 4*(lane/32) + e%4, column lane%32 of each tile
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn + j * 32 + (lane & 31);
      const float bv = (bias && EPI != kEpiDSilu) ? bias[col] : 0.0f;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int row = m0 + wm + i * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
        const size_t o = size_t(row) * ldc + col;
        const float v = acc[i][j][e];
        if constexpr (EPI == kEpiF32) {
          Cf[o] = v + bv;
        } else if constexpr (EPI == kEpiBiasSilu) {
          const float z = v + bv;
          Cf[o] = z;
          Ch[o] = __bf16(silu_f(z));
        } else if constexpr (EPI == kEpiDSilu) {
          Ch[o] = __bf16(v * dsilu_f(Zin[o]));
        } else {
          Ch[o] = __bf16(v + bv);
        }
      }
    }
}

// ------------------------------------------------------------------------------------
// MSE loss: dY = bf16(2 (Y - T) / count), per-block partial sums of (Y - T)^2 in FP64
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ Y, const float* __restrict__ T,
                                             __bf16* __restrict__ dY, int64_t n, double inv_count,
                                             double* __restrict__ partial) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const float d = Y[i] - T[i];
    s += double(d) * d;
    dY[i] = __bf16(float(2.0 * inv_count) * d);
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1] + red[2] + red[3]) * inv_count;
}

__global__ void k_sum_partials(const double* __restrict__ partial, int n, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += partial[i];
    *out = s;
  }
}

// column sums of a [rows x cols] bf16 matrix (bias gradients), FP32 accumulation
__global__ __launch_bounds__(256) void k_colsum(const __bf16* __restrict__ X, int rows, int cols,
                                                float* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float s = 0.0f;
  for (int r = 0; r < rows; ++r) s += float(X[size_t(r) * cols + c]);
  out[c] = s;
}

// Adam on FP32 master parameters with a BF16 copy for the GEMMs (bias tensors: no copy)
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                                              const float* __restrict__ g, __bf16* __restrict__ p16, int64_t n,
                                              float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pi;
  if (p16) p16[i] = __bf16(pi);
}

// ------------------------------------------------------------------------------------
// Features: the lowest modes k in [-mh, mh-1]^3 of fhat / fhat(0) (real, imaginary
// interleaved, bf16, k_z fastest) from the spectral path's half-plane fhat layout
// [row][pencil], row = kz + n/2; and rho = fhat(0) * (2L)^3 per cell.
template <typename T>
__global__ __launch_bounds__(256) void k_lowmodes(const T* __restrict__ fhat_ri, int rows, int half, int npair, int K,
                                                  int Kh, int mh, double box3, __bf16* __restrict__ X, int ldx,
                                                  float* __restrict__ rho) {
  const int cell = blockIdx.x;
  const T* fh = fhat_ri + size_t(cell) * rows * npair * 2;
  const int m = 2 * mh;
  // fhat(0): pencil (0, 0) is p = Kh*K, row n/2
  const T f0r = fh[(size_t(half) * npair + Kh * K) * 2];
  const double inv = f0r != T(0) ? 1.0 / double(f0r) : 0.0;
  if (threadIdx.x == 0) rho[cell] = float(double(f0r) * box3);
  for (int i = threadIdx.x; i < m * m * m; i += blockDim.x) {
    const int kx = i / (m * m) - mh, ky = (i / m) % m - mh, kz = i % m - mh;
    // half plane: kx > 0, or kx == 0 and ky >= 0; otherwise use the conjugate of (-k)
    const bool direct = kx > 0 || (kx == 0 && ky >= 0);
    const int ax = direct ? kx : -kx, ay = direct ? ky : -ky, az = direct ? kz : -kz;
    const int p = ax > 0 ? (ax - 1) * K + (ay + Kh) : Kh * K + ay;
    const size_t e = (size_t(az + half) * npair + p) * 2;
    // (-1)^(kx+ky+kz): the grid starts at v = -L, so the coefficient of exp(i xi.v) is the
    // index-space DFT times exp(i pi (kx+ky+kz))
    const double sg = ((kx + ky + kz) & 1) ? -1.0 : 1.0;
    const double re = sg * double(fh[e]) * inv, im = sg * double(fh[e + 1]) * inv * (direct ? 1.0 : -1.0);
    X[size_t(cell) * ldx + 2 * i] = __bf16(float(re));
    X[size_t(cell) * ldx + 2 * i + 1] = __bf16(float(im));
  }
}

// Surrogate output to Q: q = scale * rho^2 * y; moment-residual indicator
// r = max_i |sum_k phi_i(v_k) q_k| / (sum_k |phi_i(v_k)| |q_k|), phi = (1, v, |v|^2/2), FP64.
__global__ __launch_bounds__(256) void k_sur_output(const float* __restrict__ Y, int ldy, const float* __restrict__ rho,
                                                    float scale, int n, double L, float* __restrict__ q,
                                                    double* __restrict__ r_out) {
  __shared__ double red[10][4];
  const int cell = blockIdx.x;
  const size_t N3 = size_t(n) * n * n;
  const double dv = 2.0 * L / n;
  const float r2 = scale * rho[cell] * rho[cell];
  double s[5] = {0, 0, 0, 0, 0}, a[5] = {0, 0, 0, 0, 0};
  for (size_t i = threadIdx.x; i < N3; i += blockDim.x) {
    const float qv = Y[size_t(cell) * ldy + i] * r2;
    q[size_t(cell) * N3 + i] = qv;
    const int x = int(i / (size_t(n) * n)), y = int((i / n) % n), z = int(i % n);
    const double vx = -L + x * dv, vy = -L + y * dv, vz = -L + z * dv;
    const double ph[5] = {1.0, vx, vy, vz, 0.5 * (vx * vx + vy * vy + vz * vz)};
    for (int k = 0; k < 5; ++k) {
      s[k] += ph[k] * qv;
      a[k] += fabs(ph[k]) * fabs(double(qv));
    }
  }
  for (int k = 0; k < 5; ++k) {
    for (int off = 32; off > 0; off >>= 1) {
      s[k] += __shfl_xor(s[k], off, 64);
      a[k] += __shfl_xor(a[k], off, 64);
    }
  }
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < 5; ++k) {
      red[k][threadIdx.x >> 6] = s[k];
      red[5 + k][threadIdx.x >> 6] = a[k];
    }
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int k = 0; k < 5; ++k) {
      const double sk = red[k][0] + red[k][1] + red[k][2] + red[k][3];
      const double ak = red[5 + k][0] + red[5 + k][1] + red[5 + k][2] + red[5 + k][3];
      r = fmax(r, fabs(sk) / (ak + 1e-300));
    }
    r_out[cell] = r;
  }
}

// Training targets t = q / (scale rho^2) (the quantity the network predicts), in place allowed
__global__ __launch_bounds__(256) void k_sur_target(const float* __restrict__ q, const float* __restrict__ rho,
                                                    float inv_scale, float* __restrict__ t, int n3) {
  const int cell = blockIdx.y;
  const float s = inv_scale / (rho[cell] * rho[cell]);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n3; i += gridDim.x * blockDim.x)
    t[size_t(cell) * n3 + i] = q[size_t(cell) * n3 + i] * s;
}

// Compaction of the cells whose indicator exceeds the threshold (or is NaN), in cell order: one
// workgroup scans the flags (cells <= 1024 * 64) and writes the list and its length.
__global__ __launch_bounds__(1024) void k_compact(const double* __restrict__ r, int cells, double thr,
                                                  int* __restrict__ list, int* __restrict__ count) {
  __shared__ int sums[1024];
  const int per = (cells + blockDim.x - 1) / blockDim.x;
  const int c0 = threadIdx.x * per;
  int mine = 0;
  for (int c = c0; c < c0 + per && c < cells; ++c) mine += !(r[c] <= thr) ? 1 : 0;  // NaN falls back
  sums[threadIdx.x] = mine;
  __syncthreads();
  for (int off = 1; off < int(blockDim.x); off <<= 1) {  // inclusive scan
    const int v = threadIdx.x >= unsigned(off) ? sums[threadIdx.x - off] : 0;
    __syncthreads();
    sums[threadIdx.x] += v;
    __syncthreads();
  }
  int pos = sums[threadIdx.x] - mine;
  for (int c = c0; c < c0 + per && c < cells; ++c)
    if (!(r[c] <= thr)) list[pos++] = c;
  if (threadIdx.x == blockDim.x - 1) *count = sums[threadIdx.x];
}

// gather / scatter whole cells (n^3 values) by a list
template <typename T>
__global__ __launch_bounds__(256) void k_gather_cells(const T* __restrict__ src, T* __restrict__ dst,
                                                      const int* __restrict__ list, int n3) {
  const int j = blockIdx.y;
  const int c = list[j];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n3; i += gridDim.x * blockDim.x)
    dst[size_t(j) * n3 + i] = src[size_t(c) * n3 + i];
}
template <typename T>
__global__ __launch_bounds__(256) void k_scatter_cells(const T* __restrict__ src, T* __restrict__ dst,
                                                       const int* __restrict__ list, int n3) {
  const int j = blockIdx.y;
  const int c = list[j];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n3; i += gridDim.x * blockDim.x)
    dst[size_t(c) * n3 + i] = src[size_t(j) * n3 + i];
}

// ------------------------------------------------------------------------------------
// launchers
hipError_t launch_gemm(int a_km, int b_kn, int epi, const void* A, const void* B, int M, int N, int K, int lda,
                       int ldb, const float* bias, float* Cf, void* Ch, const float* Zin, int ldc, void* stream) {
  const dim3 grid(N / GBN, M / GBM);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const __bf16* a = static_cast<const __bf16*>(A);
  const __bf16* b = static_cast<const __bf16*>(B);
  __bf16* ch = static_cast<__bf16*>(Ch);
#define GEMM_CASE(AK, BK, E)                                                                             \
  if (a_km == AK && b_kn == BK && epi == E) {                                                            \
    hipLaunchKernelGGL((k_gemm<AK, BK, E>), grid, dim3(256), 0, st, a, b, M, N, K, lda, ldb, bias, Cf, ch, \
                       Zin, ldc);                                                                        \
    return hipGetLastError();                                                                            \
  }
  GEMM_CASE(false, false, kEpiF32)
  GEMM_CASE(false, false, kEpiBiasSilu)
  GEMM_CASE(false, false, kEpiBiasBf16)
  GEMM_CASE(false, true, kEpiDSilu)
  GEMM_CASE(false, true, kEpiF32)
  GEMM_CASE(true, true, kEpiF32)
#undef GEMM_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_mse(const float* Y, const float* T, void* dY, int64_t n, double* partial, int blocks,
                      void* stream) {
  hipLaunchKernelGGL(k_mse, dim3(blocks), dim3(256), 0, static_cast<hipStream_t>(stream), Y, T,
                     static_cast<__bf16*>(dY), n, 1.0 / double(n), partial);
  return hipGetLastError();
}

hipError_t launch_sum_partials(const double* partial, int n, double* out, void* stream) {
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream), partial, n, out);
  return hipGetLastError();
}

hipError_t launch_colsum(const void* X, int rows, int cols, float* out, void* stream) {
  hipLaunchKernelGGL(k_colsum, dim3((cols + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream),
                     static_cast<const __bf16*>(X), rows, cols, out);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, float* m, float* v, const float* g, void* p16, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, void* stream) {
  hipLaunchKernelGGL(k_adam, dim3(unsigned((n + 255) / 256)), dim3(256), 0, static_cast<hipStream_t>(stream), p, m, v,
                     g, static_cast<__bf16*>(p16), n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_lowmodes(int dtype_is_f32, const void* fhat, int rows, int half, int npair, int K, int Kh, int mh,
                           double box3, void* X, int ldx, float* rho, int64_t cells, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dtype_is_f32)
    hipLaunchKernelGGL(k_lowmodes<float>, dim3(unsigned(cells)), dim3(256), 0, st, static_cast<const float*>(fhat),
                       rows, half, npair, K, Kh, mh, box3, static_cast<__bf16*>(X), ldx, rho);
  else
    hipLaunchKernelGGL(k_lowmodes<double>, dim3(unsigned(cells)), dim3(256), 0, st,
                       static_cast<const double*>(fhat), rows, half, npair, K, Kh, mh, box3, static_cast<__bf16*>(X),
                       ldx, rho);
  return hipGetLastError();
}

hipError_t launch_sur_output(const float* Y, int ldy, const float* rho, float scale, int n, double L, float* q,
                             double* r, int64_t cells, void* stream) {
  hipLaunchKernelGGL(k_sur_output, dim3(unsigned(cells)), dim3(256), 0, static_cast<hipStream_t>(stream), Y, ldy, rho,
                     scale, n, L, q, r);
  return hipGetLastError();
}

hipError_t launch_sur_target(const float* q, const float* rho, float inv_scale, float* t, int n3, int64_t cells,
                             void* stream) {
  // grid.y is limited to 65535: launch in slices of cells
  for (int64_t c0 = 0; c0 < cells; c0 += 32768) {
    const int64_t c = cells - c0 < 32768 ? cells - c0 : 32768;
    const dim3 grid(unsigned((n3 + 255) / 256 < 32 ? (n3 + 255) / 256 : 32), unsigned(c));
    hipLaunchKernelGGL(k_sur_target, grid, dim3(256), 0, static_cast<hipStream_t>(stream), q + c0 * n3, rho + c0,
                       inv_scale, t + c0 * n3, n3);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_compact(const double* r, int cells, double thr, int* list, int* count, void* stream) {
  hipLaunchKernelGGL(k_compact, dim3(1), dim3(1024), 0, static_cast<hipStream_t>(stream), r, cells, thr, list, count);
  return hipGetLastError();
}

hipError_t launch_gather_cells(int scatter, const float* src, float* dst, const int* list, int count, int n3,
                               void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  // list entry j moves between src/dst cell list[j] and packed slot j; slices of 32768
  // entries keep grid.y within its limit
  for (int j0 = 0; j0 < count; j0 += 32768) {
    const int c = count - j0 < 32768 ? count - j0 : 32768;
    const dim3 grid(unsigned((n3 + 255) / 256 < 64 ? (n3 + 255) / 256 : 64), unsigned(c));
    if (scatter)
      hipLaunchKernelGGL(k_scatter_cells<float>, grid, dim3(256), 0, st, src + size_t(j0) * n3, dst, list + j0, n3);
    else
      hipLaunchKernelGGL(k_gather_cells<float>, grid, dim3(256), 0, st, src, dst + size_t(j0) * n3, list + j0, n3);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace fks
