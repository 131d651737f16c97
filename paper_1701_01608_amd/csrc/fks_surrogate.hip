// Fourier-mode MLP surrogate of the collision operator (not part of the paper): BF16
// MFMA GEMMs with FP32 accumulation for training and inference, fused bias/SiLU
// epilogues, MSE loss, Adam, the low-mode feature extraction from the spectral path's
// fhat, and the moment-residual indicator with fallback compaction.
//
// GEMM: C[M x N] = A[M x K] . B[K x N] on v_mfma_f32_32x32x16_bf16.  Operand layouts:
// A is "MK" (row-major, K contiguous) or "KM" (K rows, M contiguous); B is "NK" (each of
// the N columns stored K-contiguous, i.e. weights [out][in]) or "KN".  Tiles of 128 x 128
// x 64 are staged through LDS K-contiguous, so one kernel serves the forward product
// (A=MK, B=NK), the input gradient (A=MK, B=KN) and the weight gradient (A=KM, B=KN).
// M, N, K must be multiples of 128, 128 and 64.
#include <hip/hip_runtime.h>

#include "fks_fft.hpp"
#include "fks_internal.hpp"

namespace fks {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int GBM = 128, GBN = 128, GBK = kGemmKStep, GPAD = 8, GLD = GBK + GPAD;  // LDS row stride (bf16)
static_assert(GBK == 64, "the tile loads below move 32 bf16 of A and of B per thread and k step");

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
  kEpiBiasBf16 = 3,   // Ch = bf16(acc + bias)
  kEpiPartial = 4     // split K: Cf[blockIdx.z][M][ldc] = partial acc
};

// epilogue of one 32 x 32 accumulator tile: lane holds rows row0 + 8 (e/4) + 4 (lane/32) +
// e%4 (e < 16) of column col
template <int EPI>
__device__ __forceinline__ void gemm_store_tile(const f32x16& a, int row0, int col, int lane,
                                                const float* __restrict__ bias, float* __restrict__ Cf,
                                                __bf16* __restrict__ Ch, const float* __restrict__ Zin, int ldc) {
  const float bv = (bias && EPI != kEpiDSilu && EPI != kEpiPartial) ? bias[col] : 0.0f;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int row = row0 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
    const size_t o = size_t(row) * ldc + col;
    const float v = a[e];
    if constexpr (EPI == kEpiF32 || EPI == kEpiPartial) {
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

template <bool A_KM, bool B_KN, int EPI>
__global__ __launch_bounds__(256) void k_gemm(const __bf16* __restrict__ A, const __bf16* __restrict__ B, int M,
                                              int N, int K, int lda, int ldb, const float* __restrict__ bias,
                                              float* __restrict__ Cf, __bf16* __restrict__ Ch,
                                              const float* __restrict__ Zin, int ldc, int k_split) {
  (void)N;  // the grid covers N exactly: the launchers require N % GBN == 0
  // two LDS stages: the global loads of k tile i+1 are in flight (in registers) while
  // the matrix cores work on tile i
  __shared__ __align__(16) __bf16 As[2][GBM * GLD];
  __shared__ __align__(16) __bf16 Bs[2][GBN * GLD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * GBM, n0 = blockIdx.x * GBN;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  f32x16 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;

  // split K: blockIdx.z takes the k range [z k_split, (z + 1) k_split)
  const int kb = blockIdx.z * k_split, ke = kb + k_split < K ? kb + k_split : K;
  if constexpr (EPI == kEpiPartial) Cf += size_t(blockIdx.z) * M * ldc;

  // per-thread share of one k tile: 4 x 16 bytes of A and of B (named registers: no
  // address is taken, so nothing goes to private memory)
  uint4 ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3;
  // K-contiguous operand: row tid/2, 32 consecutive k; M- or N-contiguous operand: k rows
  // tid/8 and tid/8 + 32, 16 consecutive columns each
  auto load_tile = [&](int k0) {
    if constexpr (!A_KM) {
      const uint4* src = reinterpret_cast<const uint4*>(A + size_t(m0 + (tid >> 1)) * lda + k0 + (tid & 1) * 32);
      ra0 = src[0];
      ra1 = src[1];
      ra2 = src[2];
      ra3 = src[3];
    } else {
      const uint4* src = reinterpret_cast<const uint4*>(A + size_t(k0 + (tid >> 3)) * lda + m0 + (tid & 7) * 16);
      const uint4* src2 = reinterpret_cast<const uint4*>(A + size_t(k0 + 32 + (tid >> 3)) * lda + m0 + (tid & 7) * 16);
      ra0 = src[0];
      ra1 = src[1];
      ra2 = src2[0];
      ra3 = src2[1];
    }
    if constexpr (!B_KN) {
      const uint4* src = reinterpret_cast<const uint4*>(B + size_t(n0 + (tid >> 1)) * ldb + k0 + (tid & 1) * 32);
      rb0 = src[0];
      rb1 = src[1];
      rb2 = src[2];
      rb3 = src[3];
    } else {
      const uint4* src = reinterpret_cast<const uint4*>(B + size_t(k0 + (tid >> 3)) * ldb + n0 + (tid & 7) * 16);
      const uint4* src2 = reinterpret_cast<const uint4*>(B + size_t(k0 + 32 + (tid >> 3)) * ldb + n0 + (tid & 7) * 16);
      rb0 = src[0];
      rb1 = src[1];
      rb2 = src2[0];
      rb3 = src2[1];
    }
  };
  // 16 consecutive bf16 of one k row scattered to 16 rows of a K-contiguous tile
  auto scatter16 = [&](unsigned short* tile, int c0, int kr, const uint4& v0, const uint4& v1) {
    const uint32_t w[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      tile[(c0 + 2 * i) * GLD + kr] = static_cast<unsigned short>(w[i] & 0xffffu);
      tile[(c0 + 2 * i + 1) * GLD + kr] = static_cast<unsigned short>(w[i] >> 16);
    }
  };
  // LDS tiles K-contiguous: As[m][k], Bs[n][k]
  auto store_tile = [&](int buf) {
    if constexpr (!A_KM) {
      uint4* dst = reinterpret_cast<uint4*>(As[buf] + (tid >> 1) * GLD + (tid & 1) * 32);
      dst[0] = ra0;
      dst[1] = ra1;
      dst[2] = ra2;
      dst[3] = ra3;
    } else {
      unsigned short* t = reinterpret_cast<unsigned short*>(As[buf]);
      scatter16(t, (tid & 7) * 16, tid >> 3, ra0, ra1);
      scatter16(t, (tid & 7) * 16, 32 + (tid >> 3), ra2, ra3);
    }
    if constexpr (!B_KN) {
      uint4* dst = reinterpret_cast<uint4*>(Bs[buf] + (tid >> 1) * GLD + (tid & 1) * 32);
      dst[0] = rb0;
      dst[1] = rb1;
      dst[2] = rb2;
      dst[3] = rb3;
    } else {
      unsigned short* t = reinterpret_cast<unsigned short*>(Bs[buf]);
      scatter16(t, (tid & 7) * 16, tid >> 3, rb0, rb1);
      scatter16(t, (tid & 7) * 16, 32 + (tid >> 3), rb2, rb3);
    }
  };

  if (kb < ke) {
    load_tile(kb);
    store_tile(0);
  }
  __syncthreads();
  int cur = 0;
  for (int k0 = kb; k0 < ke; k0 += GBK) {
    const bool more = k0 + GBK < ke;
    if (more) load_tile(k0 + GBK);
#pragma unroll
    for (int kk = 0; kk < GBK; kk += 16) {
      bf16x8 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a[i] = *reinterpret_cast<const bf16x8*>(As[cur] + (wm + i * 32 + (lane & 31)) * GLD + kk + 8 * (lane >> 5));
        b[i] = *reinterpret_cast<const bf16x8*>(Bs[cur] + (wn + i * 32 + (lane & 31)) * GLD + kk + 8 * (lane >> 5));
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) store_tile(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
  // ---- epilogue
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
      gemm_store_tile<EPI>(acc[i][j], m0 + wm + i * 32, n0 + wn + j * 32 + (lane & 31), lane, bias, Cf, Ch, Zin, ldc);
}

// Large-tile GEMM for K-contiguous A and B (A = MK, B = NK): 256 x 256 x 64 block tiles,
// four waves of 128 x 128 (sixteen 32 x 32 accumulators each), two LDS stages of 72 KiB.
// Each block moves 64 KiB per k step for 8.4 MFLOP (128 flop per byte from L2, twice the
// 128 x 128 tile), which the large products of the output layer need.  M, N multiples of
// 256, K (and the split-K range) multiples of 64.
constexpr int BBM = 256, BBN = 256;
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm_big(const __bf16* __restrict__ A, const __bf16* __restrict__ B, int M,
                                                  int N, int K, int lda, int ldb, const float* __restrict__ bias,
                                                  float* __restrict__ Cf, __bf16* __restrict__ Ch,
                                                  const float* __restrict__ Zin, int ldc, int k_split) {
  (void)N;  // the grid covers N exactly: the launchers require N % BBN == 0
  __shared__ __align__(16) __bf16 smem[2][(BBM + BBN) * GLD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * BBM, n0 = blockIdx.x * BBN;
  const int wm = (wave >> 1) * 128, wn = (wave & 1) * 128;
  f32x16 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;
  const int kb = blockIdx.z * k_split, ke = kb + k_split < K ? kb + k_split : K;
  if constexpr (EPI == kEpiPartial) Cf += size_t(blockIdx.z) * M * ldc;

  // per thread and k step: rows tid/8 + 32 j (j < 8) of A and of B, 8 bf16 at k offset 8 (tid%8);
  // the staging arrays are indexed by compile-time constants only, so they stay in registers
  u32x4 ra[8], rb[8];
  // uniform row bases plus one 32-bit lane offset per operand (scalar-base addressing)
  const unsigned va = unsigned(((tid >> 3) * lda + (tid & 7) * 8) * 2);
  const unsigned vb = unsigned(((tid >> 3) * ldb + (tid & 7) * 8) * 2);
  const int st_off = (tid >> 3) * GLD + (tid & 7) * 8;
#define GEMM_BIG_LOAD(k0)                                                                        \
  static_for<0, 8>([&](auto jj) {                                                                \
    constexpr int j = decltype(jj)::value;                                                       \
    const char* a_row = reinterpret_cast<const char*>(A + size_t(m0 + 32 * j) * lda + (k0));     \
    const char* b_row = reinterpret_cast<const char*>(B + size_t(n0 + 32 * j) * ldb + (k0));     \
    ra[j] = *reinterpret_cast<const u32x4*>(a_row + va);                                         \
    rb[j] = *reinterpret_cast<const u32x4*>(b_row + vb);                                         \
  });
#define GEMM_BIG_STORE(buf)                                                             \
  static_for<0, 8>([&](auto jj) {                                                       \
    constexpr int j = decltype(jj)::value;                                              \
    *reinterpret_cast<u32x4*>(smem[buf] + st_off + 32 * j * GLD) = ra[j];               \
    *reinterpret_cast<u32x4*>(smem[buf] + BBM * GLD + st_off + 32 * j * GLD) = rb[j];   \
  });

  if (kb < ke) {
    GEMM_BIG_LOAD(kb)
    GEMM_BIG_STORE(0)
  }
  __syncthreads();
  int cur = 0;
  for (int k0 = kb; k0 < ke; k0 += GBK) {
    if (k0 + GBK < ke) {
      GEMM_BIG_LOAD(k0 + GBK)
    }
    sched_fence();
    const __bf16* As = smem[cur] + (wm + (lane & 31)) * GLD + 8 * (lane >> 5);
    const __bf16* Bs = smem[cur] + BBM * GLD + (wn + (lane & 31)) * GLD + 8 * (lane >> 5);
    // fragments double-buffered in registers: the reads of k sub-step q + 1 are issued
    // between the sixteen products of sub-step q (one read per two products); during the
    // last sub-step the staged next tile is written to the other LDS stage instead (also
    // after the final tile, where it rewrites data nobody reads: no branch in the schedule)
    bf16x8 fa[2][4], fb[2][4];
    static_for<0, 4>([&](auto ii) {
      constexpr int r = decltype(ii)::value;
      fa[0][r] = *reinterpret_cast<const bf16x8*>(As + r * 32 * GLD);
      fb[0][r] = *reinterpret_cast<const bf16x8*>(Bs + r * 32 * GLD);
    });
    static_for<0, GBK / 16>([&](auto qq) {
      constexpr int q = decltype(qq)::value, c = q & 1;
      if constexpr (q + 1 < GBK / 16) {
        static_for<0, 4>([&](auto ii) {
          constexpr int r = decltype(ii)::value;
          fa[c ^ 1][r] = *reinterpret_cast<const bf16x8*>(As + r * 32 * GLD + (q + 1) * 16);
          fb[c ^ 1][r] = *reinterpret_cast<const bf16x8*>(Bs + r * 32 * GLD + (q + 1) * 16);
        });
      } else {
        GEMM_BIG_STORE(cur ^ 1)
      }
      static_for<0, 4>([&](auto ii) {
        static_for<0, 4>([&](auto jj) {
          constexpr int r = decltype(ii)::value, t = decltype(jj)::value;
          acc[r][t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[c][r], fb[c][t], acc[r][t], 0, 0, 0);
        });
      });
      if constexpr (q + 1 < GBK / 16) {
        static_for<0, 8>([&](auto) {
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // one LDS read
          __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);  // two MFMA
        });
      } else {
        static_for<0, 16>([&](auto) {
          __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);  // one LDS write
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
        });
      }
      sched_fence();
    });
    __syncthreads();
    cur ^= 1;
  }
#undef GEMM_BIG_LOAD
#undef GEMM_BIG_STORE
  static_for<0, 4>([&](auto ii) {
    static_for<0, 4>([&](auto jj) {
      constexpr int r = decltype(ii)::value, t = decltype(jj)::value;
      gemm_store_tile<EPI>(acc[r][t], m0 + wm + r * 32, n0 + wn + t * 32 + (lane & 31), lane, bias, Cf, Ch, Zin, ldc);
      sched_fence();  // one accumulator tile at a time: bounded register use
    });
  });
}

// split-K reduction with the input-gradient epilogue: Ch = bf16(sum_z P[z] * silu'(Zin))
__global__ __launch_bounds__(256) void k_splitk_dsilu(const float* __restrict__ Pz, int splits, int64_t mn,
                                                      const float* __restrict__ Zin, __bf16* __restrict__ Ch) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < mn; i += int64_t(gridDim.x) * blockDim.x) {
    float a = 0.0f;
    for (int z = 0; z < splits; ++z) a += Pz[size_t(z) * mn + i];
    Ch[i] = __bf16(a * dsilu_f(Zin[i]));
  }
}

// ------------------------------------------------------------------------------------
// MSE loss: dY = bf16(2 (Y - T) / count), per-block partial sums of (Y - T)^2 in FP64;
// four elements per thread and step (n is a multiple of 4)
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ Y, const float* __restrict__ T,
                                             __bf16* __restrict__ dY, int64_t n, double inv_count,
                                             double* __restrict__ partial) {
  __shared__ double red[4];
  double s = 0.0;
  const float sc = float(2.0 * inv_count);
  const int64_t n4 = n >> 2;
  const float4* Y4 = reinterpret_cast<const float4*>(Y);
  const float4* T4 = reinterpret_cast<const float4*>(T);
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n4; i += int64_t(gridDim.x) * blockDim.x) {
    const float4 y = Y4[i], t = T4[i];
    const float d0 = y.x - t.x, d1 = y.y - t.y, d2 = y.z - t.z, d3 = y.w - t.w;
    s += double(d0 * d0 + d1 * d1) + double(d2 * d2 + d3 * d3);
    __bf16* o = dY + 4 * i;
    o[0] = __bf16(sc * d0);
    o[1] = __bf16(sc * d1);
    o[2] = __bf16(sc * d2);
    o[3] = __bf16(sc * d3);
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1] + red[2] + red[3]) * inv_count;
}

// sum of n partials by one workgroup of 256 threads (tree over the waves)
__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ partial, int n,
                                                      double* __restrict__ out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += partial[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = (red[0] + red[1]) + (red[2] + red[3]);
}

// out[c][r] = in[r][c] for a [rows][cols] bf16 matrix (64 x 64 tiles through LDS)
__global__ __launch_bounds__(256) void k_transpose_bf16(const unsigned short* __restrict__ in, int rows, int cols,
                                                        unsigned short* __restrict__ out) {
  __shared__ unsigned short tile[64][65];
  const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int i = ty; i < 64; i += 4) tile[i][tx] = in[size_t(r0 + i) * cols + c0 + tx];
  __syncthreads();
  for (int i = ty; i < 64; i += 4) out[size_t(c0 + i) * rows + r0 + tx] = tile[tx][i];
}

// column sums of a [rows x cols] bf16 matrix (bias gradients), FP32 accumulation, in two
// passes: row block y of each column into partial[y][col], then the sum over blocks
__global__ __launch_bounds__(256) void k_colsum_part(const __bf16* __restrict__ X, int rows, int cols, int rows_per,
                                                     float* __restrict__ partial) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  const int r0 = blockIdx.y * rows_per, r1 = r0 + rows_per < rows ? r0 + rows_per : rows;
  float s = 0.0f;
  for (int r = r0; r < r1; ++r) s += float(X[size_t(r) * cols + c]);
  partial[size_t(blockIdx.y) * cols + c] = s;
}
__global__ __launch_bounds__(256) void k_colsum_final(const float* __restrict__ partial, int blocks, int cols,
                                                      float* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float s = 0.0f;
  for (int y = 0; y < blocks; ++y) s += partial[size_t(y) * cols + c];
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
                                                  float* __restrict__ rho, const double* __restrict__ mom, double L) {
  const int cell = blockIdx.x;
  // centring: the coefficients of f(v + u), u the cell's mean velocity, are fhat_k e^{i xi_k.u}
  double ux = 0.0, uy = 0.0, uz = 0.0;
  if (mom) {
    const double m0 = mom[size_t(cell) * 5];
    ux = mom[size_t(cell) * 5 + 1] / m0;
    uy = mom[size_t(cell) * 5 + 2] / m0;
    uz = mom[size_t(cell) * 5 + 3] / m0;
  }
  const double wq = 3.14159265358979323846 / L;
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
    double re = sg * double(fh[e]) * inv, im = sg * double(fh[e + 1]) * inv * (direct ? 1.0 : -1.0);
    if (mom) {
      double sn, cs;
      sincos(wq * (kx * ux + ky * uy + kz * uz), &sn, &cs);
      const double r2 = re * cs - im * sn, i2 = re * sn + im * cs;
      re = r2;
      im = i2;
    }
    X[size_t(cell) * ldx + 2 * i] = __bf16(float(re));
    X[size_t(cell) * ldx + 2 * i + 1] = __bf16(float(im));
  }
}

__device__ __forceinline__ void block_reduce_moments(double (&v)[5], double* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  for (int i = 0; i < 5; ++i) {
    double x = v[i];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) red[i * 16 + wid] = x;
  }
  __syncthreads();
  for (int i = 0; i < 5; ++i) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += red[i * 16 + w];
    v[i] = t;
  }
}

// Pruned feature transform: only the lowest modes k in [-MH, MH-1]^3 of f, by direct
// separable sums with compile-time twiddles (z: the N real samples of a row against
// k_z = 0..MH, the negative k_z by conjugation; then y and x over the complex partials),
// reading f once.  The same pass forms the FP64 moments sum phi f dv^3 of the cell, from
// which rho and (centring) the mean velocity u follow.  Output as k_lowmodes.
template <typename T, int N, int MH>
__global__ __launch_bounds__(256) void k_features(const T* __restrict__ f, __bf16* __restrict__ X, int ldx,
                                                  float* __restrict__ rho_out, double* __restrict__ mom_out,
                                                  int center, double L) {
  constexpr int M = 2 * MH;
  static_assert(MH <= N / 2 - 1, "modes beyond the kept set");
  static_assert(N * M <= 256, "one y line per thread");
  static_assert(M * M <= N * (MH + 1), "y partials fit in the z partials' storage");
  __shared__ cpx<float> zs[N * N][MH + 1];  // z partials [x][y][kz], kz = 0..MH (negative kz: conjugates)
  // y partials [x][ky + MH][kz + MH], in the same storage once every z partial has been read
  cpx<float>(*ys)[M][M] = reinterpret_cast<cpx<float>(*)[M][M]>(&zs[0][0]);
  __shared__ double red[5 * 16];
  const int cell = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  const T* fc = f + size_t(cell) * N * N * N;
  const double dv = 2.0 * L / N;
  // index moments (FP64, literal integer weights): sum f, sum i f, sum j f, sum k f,
  // sum (i^2 + j^2 + k^2) f over grid indices; the velocity moments follow after the
  // block sum from v = -L + index dv
  double m[5] = {0, 0, 0, 0, 0};
  // z pass + moments
  for (int row = tid; row < N * N; row += nt) {
    T r[N];
    static_for<0, N>([&](auto z) { r[z] = fc[size_t(row) * N + decltype(z)::value]; });
    double s0 = 0, sz = 0, szz = 0;
    static_for<0, N>([&](auto z) {
      constexpr double iz = double(decltype(z)::value);
      const double d = double(r[z]);
      s0 += d;
      sz += iz * d;
      szz += (iz * iz) * d;
      if constexpr (decltype(z)::value % 8 == 7) sched_fence();
    });
    const double ix = double(row / N), iy = double(row % N);
    m[0] += s0;
    m[1] += ix * s0;
    m[2] += iy * s0;
    m[3] += sz;
    m[4] += (ix * ix + iy * iy) * s0 + szz;
    static_for<0, MH + 1>([&](auto kk) {
      constexpr int k = decltype(kk)::value;
      float re = 0.0f, im = 0.0f;
      static_for<0, N>([&](auto z) {
        constexpr sc w = sincos2pi(-long(k) * decltype(z)::value, N);  // e^{-2 pi i k z / N}
        if constexpr (w.c != 0.0) re += float(w.c) * float(r[z]);
        if constexpr (w.s != 0.0) im += float(w.s) * float(r[z]);
      });
      zs[row][k] = cpx<float>{re, im};
      sched_fence();
    });
  }
  // y pass: lines (x, kz)
  __syncthreads();
  cpx<float> acc[M];
  static_for<0, M>([&](auto k) { acc[k] = cpx<float>{0.0f, 0.0f}; });
  if (tid < N * M) {
    const int x = tid / M, kzi = tid % M;
    const int kz = kzi - MH, kza = kz < 0 ? -kz : kz;
    const float cs = kz < 0 ? -1.0f : 1.0f;  // f real: the kz < 0 partial is the conjugate
    static_for<0, N>([&](auto yy) {
      constexpr int y = decltype(yy)::value;
      const cpx<float> zv = zs[x * N + y][kza];
      const cpx<float> v = {zv.re, cs * zv.im};
      static_for<0, M>([&](auto kk) {
        constexpr sc w = sincos2pi(-long(decltype(kk)::value - MH) * y, N);
        acc[kk] = acc[kk] + cmul(v, cpx<float>{float(w.c), float(w.s)});
      });
      if constexpr (y % 8 == 7) sched_fence();
    });
  }
  __syncthreads();  // every z partial read: the storage now takes the y partials
  if (tid < N * M) static_for<0, M>([&](auto k) { ys[tid / M][decltype(k)::value][tid % M] = acc[k]; });
  block_reduce_moments(m, red);
  __syncthreads();
  {
    const double a0 = m[0], ax = m[1], ay = m[2], az = m[3], b = m[4];
    m[1] = -L * a0 + dv * ax;
    m[2] = -L * a0 + dv * ay;
    m[3] = -L * a0 + dv * az;
    m[4] = 0.5 * (3.0 * L * L * a0 - 2.0 * L * dv * (ax + ay + az) + dv * dv * b);
  }
  const double S = m[0];  // sum of f over the grid
  const double inv = S != 0.0 ? 1.0 / S : 0.0;
  double ux = 0, uy = 0, uz = 0;
  if (S != 0.0) {
    ux = m[1] / S;
    uy = m[2] / S;
    uz = m[3] / S;
  }
  if (tid == 0) {
    const double w3 = dv * dv * dv;
    rho_out[cell] = float(S * w3);
    if (mom_out)
      for (int i = 0; i < 5; ++i) mom_out[size_t(cell) * 5 + i] = m[i] * w3;
  }
  // x pass: lines (ky, kz) -> kx; normalise, grid-origin and centring phases, bf16
  const double wq = 3.14159265358979323846 / L;
  for (int it = tid; it < M * M; it += nt) {
    const int kyi = it / M, kzi = it % M;
    const int ky = kyi - MH, kz = kzi - MH;
    cpx<float> acc[M];
    static_for<0, M>([&](auto k) { acc[k] = cpx<float>{0.0f, 0.0f}; });
    static_for<0, N>([&](auto xx) {
      constexpr int x = decltype(xx)::value;
      const cpx<float> v = ys[x][kyi][kzi];
      static_for<0, M>([&](auto kk) {
        constexpr sc w = sincos2pi(-long(decltype(kk)::value - MH) * x, N);
        acc[kk] = acc[kk] + cmul(v, cpx<float>{float(w.c), float(w.s)});
      });
      if constexpr (x % 8 == 7) sched_fence();
    });
    // centring phase exp(i wq k.u), advanced along kx by repeated FP64 rotation
    double pc = 1.0, ps = 0.0, sc_ = 1.0, ss_ = 0.0;
    if (center) {
      sincos(wq * (-MH * ux + ky * uy + kz * uz), &ps, &pc);
      sincos(wq * ux, &ss_, &sc_);
    }
    static_for<0, M>([&](auto kk) {
      constexpr int kx = decltype(kk)::value - MH;
      double re = double(acc[kk].re) * inv, im = double(acc[kk].im) * inv;
      if ((kx + ky + kz) & 1) {
        re = -re;
        im = -im;
      }
      const double r2 = re * pc - im * ps, i2 = re * ps + im * pc;
      re = r2;
      im = i2;
      const double pc2 = pc * sc_ - ps * ss_, ps2 = pc * ss_ + ps * sc_;
      pc = pc2;
      ps = ps2;
      const int i = (decltype(kk)::value * M + kyi) * M + kzi;
      X[size_t(cell) * ldx + 2 * i] = __bf16(float(re));
      X[size_t(cell) * ldx + 2 * i + 1] = __bf16(float(im));
    });
  }
}

// Surrogate output to Q: q = scale * rho^2 * y; moment-residual indicator
// r = max_i |sum_k phi_i(v_k) q_k| / (sum_k |phi_i(v_k)| |q_k|), phi = (1, v, |v|^2/2), FP64.
__global__ __launch_bounds__(256) void k_sur_output(const float* __restrict__ Y, int ldy, const float* __restrict__ rho,
                                                    float scale, int n, double L, float* __restrict__ q,
                                                    double* __restrict__ r_out, int absolute) {
  __shared__ double red[10][4];
  __shared__ double rq2[4];
  const int cell = blockIdx.x;
  const size_t N3 = size_t(n) * n * n;
  const double dv = 2.0 * L / n;
  const float r2 = scale * rho[cell] * rho[cell];
  double s[5] = {0, 0, 0, 0, 0}, a[5] = {0, 0, 0, 0, 0}, q2 = 0.0;
  for (size_t i = threadIdx.x; i < N3; i += blockDim.x) {
    const float qv = Y[size_t(cell) * ldy + i] * r2;
    q[size_t(cell) * N3 + i] = qv;
    q2 += double(qv) * double(qv);
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
  for (int off = 32; off > 0; off >>= 1) q2 += __shfl_xor(q2, off, 64);
  if ((threadIdx.x & 63) == 0) {
    for (int k = 0; k < 5; ++k) {
      red[k][threadIdx.x >> 6] = s[k];
      red[5 + k][threadIdx.x >> 6] = a[k];
    }
    rq2[threadIdx.x >> 6] = q2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int k = 0; k < 5; ++k) {
      const double sk = red[k][0] + red[k][1] + red[k][2] + red[k][3];
      const double ak = red[5 + k][0] + red[5 + k][1] + red[5 + k][2] + red[5 + k][3];
      r = fmax(r, fabs(sk) / (ak + 1e-300));
    }
    if (absolute) r *= sqrt(rq2[0] + rq2[1] + rq2[2] + rq2[3]);
    r_out[cell] = r;
  }
}

// Spectral shift of whole cells: out(v) = m_c in(v + sign u_c) on the velocity grid, u_c the
// cell's mean velocity (moments mom[c] = sum phi f dv^3), m_c = 1, scale rho_c^2 or
// 1 / (scale rho_c^2) for mode 0, 1, 2.  The shift of the Fourier interpolant (Nyquist
// modes dropped, as everywhere in the method) factorises over the axes, so it is three
// passes of real 1-D line shifts (real DFT, phase e^{i pi k delta / L}, Hermitian inverse
// DFT) on the cell held in LDS.  Optionally the moment-residual indicator of the output.
constexpr int gcd_(int a, int b) { return b == 0 ? a : gcd_(b, a % b); }

template <int N>
struct ShiftLds {
  static constexpr int RS = N + 1;  // padded z row (floats)
  static constexpr int KH1 = N / 2;
  static constexpr size_t data_bytes = size_t(N) * N * RS * sizeof(float);
  static constexpr size_t bytes = data_bytes + 3 * KH1 * sizeof(cpx<float>);
  static constexpr int TPB = (512 / (N * 64 / gcd_(N, 64))) * (N * 64 / gcd_(N, 64));  // threads per block
  static_assert(bytes <= 156 * 1024, "cell does not fit in LDS");
};

__device__ __forceinline__ void block_sum11(double (&v)[11], double* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int i = 0; i < 11; ++i) {
    double x = v[i];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) red[i * 16 + wid] = x;
  }
  __syncthreads();
  for (int i = 0; i < 11; ++i) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += red[i * 16 + w];
    v[i] = t;
  }
}

// one real line shift in registers: r (N samples) -> r (N samples of the shifted
// interpolant), phase table ph (k = 0..N/2-1, 1/N of the inverse included)
template <int N>
__device__ __forceinline__ void shift_line(float* r, const cpx<float>* ph) {
  constexpr int M = N / 2;
  cpx<float> o[M];
  rdft_low<N, M>(r, o);
  static_for<0, M>([&](auto k) { o[k] = cmul(o[k], ph[decltype(k)::value]); });
  // real inverse from the Hermitian half (Nyquist zero) by one N/2-point complex DFT:
  // z_j = x_{2j} + i x_{2j+1} = sum_k (X_k + conj X_{M-k} + i (X_k - conj X_{M-k}) w^k) e^{2 pi i jk/M}
  cpx<float> z[M];
  static_for<0, M>([&](auto k) {
    constexpr int kk = decltype(k)::value;
    cpx<float> xk = {o[0].re, 0.0f}, xm = {0.0f, 0.0f};  // X_k and conj X_{M-k}, X_M = 0
    if constexpr (kk > 0) {
      xk = o[kk];
      xm = conj(o[M - kk]);
    }
    const cpx<float> sp = xk + xm, dm = twiddle<N, +1, kk>(xk - xm);
    z[kk] = cpx<float>{sp.re - dm.im, sp.im + dm.re};
  });
  dft<M, +1>(z);
  static_for<0, M>([&](auto j) {
    r[2 * decltype(j)::value] = z[j].re;
    r[2 * decltype(j)::value + 1] = z[j].im;
  });
}

template <int N>
__global__ __launch_bounds__(512) void k_shift(const float* __restrict__ in, int64_t ld_in, float* __restrict__ out,
                                               const double* __restrict__ mom, int sign, double L,
                                               const float* __restrict__ rho, float scale, int mode,
                                               double* __restrict__ r_out, int absolute) {
  using SL = ShiftLds<N>;
  constexpr int RS = SL::RS, KH1 = SL::KH1;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ double red[11 * 16];
  float* sm = reinterpret_cast<float*>(lds_raw);
  cpx<float>* ph = reinterpret_cast<cpx<float>*>(lds_raw + SL::data_bytes);
  const int cell = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  const double m0 = mom[size_t(cell) * 5];
  const double u[3] = {mom[size_t(cell) * 5 + 1] / m0, mom[size_t(cell) * 5 + 2] / m0, mom[size_t(cell) * 5 + 3] / m0};
  float mult = 1.0f;
  if (mode == 1) mult = scale * rho[cell] * rho[cell];
  if (mode == 2) mult = 1.0f / (scale * rho[cell] * rho[cell]);
  // phase tables e^{i pi k sign u_a / L}, k = 0..N/2-1, with the 1/N of the inverse DFT
  for (int i = tid; i < 3 * KH1; i += nt) {
    const int a = i / KH1, k = i % KH1;
    double sn, cs;
    sincos(double(sign) * 3.14159265358979323846 * k * u[a] / L, &sn, &cs);
    ph[i] = cpx<float>{float(cs / N), float(sn / N)};
  }
  __syncthreads();
  // the cell into LDS by coalesced 16-byte loads (consecutive lanes, consecutive float4;
  // all of a thread's loads in flight at once), rows (x, y) of N floats at stride RS
  const float4* ic4 = reinterpret_cast<const float4*>(in + size_t(cell) * ld_in);
  constexpr int NV = N * N * N / 4;  // float4 per cell
  constexpr int NR = (NV + SL::TPB - 1) / SL::TPB;  // rounds (the last may be partial)
  {
    float4 v[NR];
    static_for<0, NR>([&](auto q) {
      const int i = tid + decltype(q)::value * SL::TPB;
      if (NV % SL::TPB == 0 || i < NV) v[q] = ic4[i];
    });
    static_for<0, NR>([&](auto q) {
      const int i = tid + decltype(q)::value * SL::TPB, row = i / (N / 4), col = 4 * (i % (N / 4));
      if (NV % SL::TPB == 0 || i < NV) {
        float* d = sm + row * RS + col;
        d[0] = v[q].x * mult;
        d[1] = v[q].y * mult;
        d[2] = v[q].z * mult;
        d[3] = v[q].w * mult;
      }
    });
  }
  __syncthreads();
  // z pass in LDS: row (x, y), in place (each row belongs to one thread)
  for (int line = tid; line < N * N; line += nt) {
    float r[N];
    static_for<0, N>([&](auto j) { r[j] = sm[line * RS + decltype(j)::value]; });
    shift_line<N>(r, ph + 2 * KH1);
    static_for<0, N>([&](auto j) { sm[line * RS + decltype(j)::value] = r[j]; });
  }
  __syncthreads();
  // y pass in LDS: lines (x, z), stride RS
  for (int line = tid; line < N * N; line += nt) {
    const int base = (line / N) * N * RS + (line % N);
    float r[N];
    static_for<0, N>([&](auto j) { r[j] = sm[base + decltype(j)::value * RS]; });
    shift_line<N>(r, ph + KH1);
    static_for<0, N>([&](auto j) { sm[base + decltype(j)::value * RS] = r[j]; });
  }
  __syncthreads();
  // x pass: lines (y, z), stride N RS in LDS; results go straight to global memory
  // (lanes hold consecutive z: coalesced) with the FP64 moment sums of the output.
  // The block size is a multiple of N, so a thread's lines share one z; per line the
  // sums over x are taken first, then weighted by v_y (and v_z once at the end).
  float* oc = out + size_t(cell) * N * N * N;
  const double dv = 2.0 * L / N;
  double s0 = 0, sx = 0, sy = 0, s2 = 0, a0 = 0, ax = 0, ay = 0, a2 = 0, qq = 0;
  for (int line = tid; line < N * N; line += nt) {
    const int y = line / N, z = line % N;
    const int base = y * RS + z;
    float r[N];
    static_for<0, N>([&](auto j) { r[j] = sm[base + decltype(j)::value * N * RS]; });
    shift_line<N>(r, ph);
    static_for<0, N>([&](auto j) { oc[(size_t(decltype(j)::value) * N + y) * N + z] = r[j]; });
    if (r_out) {
      double l0 = 0, l1 = 0, l2 = 0, b0 = 0, b1 = 0, b2 = 0;
      static_for<0, N>([&](auto j) {
        const double vx = -L + decltype(j)::value * dv, d = double(r[j]), ad = fabs(d);
        qq += d * d;
        l0 += d;
        l1 += vx * d;
        l2 += vx * vx * d;
        b0 += ad;
        b1 += fabs(vx) * ad;
        b2 += vx * vx * ad;
      });
      const double vy = -L + y * dv;
      s0 += l0;
      sx += l1;
      sy += vy * l0;
      s2 += l2 + vy * vy * l0;
      a0 += b0;
      ax += b1;
      ay += fabs(vy) * b0;
      a2 += b2 + vy * vy * b0;
    }
  }
  if (r_out) {
    const double vz = -L + (tid % N) * dv;
    double acc[11] = {s0, sx, sy, vz * s0, 0.5 * (s2 + vz * vz * s0),
                      a0, ax, ay, fabs(vz) * a0, 0.5 * (a2 + vz * vz * a0), qq};
    block_sum11(acc, red);
    if (tid == 0) {
      double rr = 0.0;
      for (int k = 0; k < 5; ++k) rr = fmax(rr, fabs(acc[k]) / (acc[5 + k] + 1e-300));
      if (absolute) rr *= sqrt(acc[10]);
      r_out[cell] = rr;
    }
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
  if (M % GBM || N % GBN || K % GBK) return hipErrorInvalidValue;
  const dim3 grid(N / GBN, M / GBM);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const __bf16* a = static_cast<const __bf16*>(A);
  const __bf16* b = static_cast<const __bf16*>(B);
  __bf16* ch = static_cast<__bf16*>(Ch);
#define GEMM_CASE(AK, BK, E)                                                                             \
  if (a_km == AK && b_kn == BK && epi == E) {                                                            \
    hipLaunchKernelGGL((k_gemm<AK, BK, E>), grid, dim3(256), 0, st, a, b, M, N, K, lda, ldb, bias, Cf, ch, \
                       Zin, ldc, K);                                                                     \
    return hipGetLastError();                                                                            \
  }
  // large K-contiguous products with enough 256 x 256 tiles to fill the chip
  if (!a_km && !b_kn && M % BBM == 0 && N % BBN == 0 && int64_t(M / BBM) * (N / BBN) >= 256 &&
      (epi == kEpiF32 || epi == kEpiBiasBf16)) {
    const dim3 gb(N / BBN, M / BBM);
    if (epi == kEpiF32)
      hipLaunchKernelGGL((k_gemm_big<kEpiF32>), gb, dim3(256), 0, st, a, b, M, N, K, lda, ldb, bias, Cf, ch, Zin, ldc, K);
    else
      hipLaunchKernelGGL((k_gemm_big<kEpiBiasBf16>), gb, dim3(256), 0, st, a, b, M, N, K, lda, ldb, bias, Cf, ch, Zin,
                         ldc, K);
    return hipGetLastError();
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

// split-K product A [M][K] (MK) . B with B "KN" ([K][N]) or, b_kn = 0, "NK" ([N][K]; then M
// and N must be multiples of 256 for the large-tile kernel), reduced with the SiLU' epilogue
hipError_t launch_gemm_dsilu_splitk(const void* A, const void* B, int b_kn, int M, int N, int K, int lda, int ldb,
                                   const float* Zin, void* Ch, int splits, float* partial, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (splits < 1 || K % (splits * GBK)) return hipErrorInvalidValue;
  const int k_split = K / splits;
  if (b_kn) {
    if (M % GBM || N % GBN) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_gemm<false, true, kEpiPartial>), dim3(N / GBN, M / GBM, splits), dim3(256), 0, st,
                       static_cast<const __bf16*>(A), static_cast<const __bf16*>(B), M, N, K, lda, ldb,
                       static_cast<const float*>(nullptr), partial, static_cast<__bf16*>(nullptr), Zin, N, k_split);
  } else {
    if (M % BBM || N % BBN) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_gemm_big<kEpiPartial>), dim3(N / BBN, M / BBM, splits), dim3(256), 0, st,
                       static_cast<const __bf16*>(A), static_cast<const __bf16*>(B), M, N, K, lda, ldb,
                       static_cast<const float*>(nullptr), partial, static_cast<__bf16*>(nullptr), Zin, N, k_split);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t mn = int64_t(M) * N;
  hipLaunchKernelGGL(k_splitk_dsilu, dim3(unsigned((mn + 255) / 256 < 4096 ? (mn + 255) / 256 : 4096)), dim3(256), 0,
                     st, partial, splits, mn, Zin, static_cast<__bf16*>(Ch));
  return hipGetLastError();
}

hipError_t launch_mse(const float* Y, const float* T, void* dY, int64_t n, double* partial, int blocks,
                      void* stream) {
  hipLaunchKernelGGL(k_mse, dim3(blocks), dim3(256), 0, static_cast<hipStream_t>(stream), Y, T,
                     static_cast<__bf16*>(dY), n, 1.0 / double(n), partial);
  return hipGetLastError();
}

hipError_t launch_sum_partials(const double* partial, int n, double* out, void* stream) {
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, static_cast<hipStream_t>(stream), partial, n, out);
  return hipGetLastError();
}

hipError_t launch_transpose_bf16(const void* in, int rows, int cols, void* out, void* stream) {
  if (rows % 64 || cols % 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_transpose_bf16, dim3(cols / 64, rows / 64), dim3(256), 0, static_cast<hipStream_t>(stream),
                     static_cast<const unsigned short*>(in), rows, cols, static_cast<unsigned short*>(out));
  return hipGetLastError();
}

hipError_t launch_colsum(const void* X, int rows, int cols, float* out, float* partial, int max_blocks,
                         void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  int blocks = (rows + 63) / 64;
  if (blocks > max_blocks) blocks = max_blocks;
  const int rows_per = (rows + blocks - 1) / blocks;
  hipLaunchKernelGGL(k_colsum_part, dim3((cols + 255) / 256, blocks), dim3(256), 0, st,
                     static_cast<const __bf16*>(X), rows, cols, rows_per, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_colsum_final, dim3((cols + 255) / 256), dim3(256), 0, st, partial, blocks, cols, out);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, float* m, float* v, const float* g, void* p16, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, void* stream) {
  hipLaunchKernelGGL(k_adam, dim3(unsigned((n + 255) / 256)), dim3(256), 0, static_cast<hipStream_t>(stream), p, m, v,
                     g, static_cast<__bf16*>(p16), n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

template <typename T, int N, int MH>
static hipError_t launch_features_n(const void* f, void* X, int ldx, float* rho, double* mom, int center, double L,
                                    int64_t cells, hipStream_t st) {
  hipLaunchKernelGGL((k_features<T, N, MH>), dim3(unsigned(cells)), dim3(256), 0, st, static_cast<const T*>(f),
                     static_cast<__bf16*>(X), ldx, rho, mom, center, L);
  return hipGetLastError();
}

// pruned feature transform for the compiled (n, modes) pairs; hipErrorNotSupported
// otherwise (the caller then takes the full transform)
hipError_t launch_features(int dtype_is_f32, int n, int modes, const void* f, void* X, int ldx, float* rho,
                           double* mom, int center, double L, int64_t cells, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
#define FEAT(T, NN, MM) \
  if (n == NN && modes == 2 * MM) return launch_features_n<T, NN, MM>(f, X, ldx, rho, mom, center, L, cells, st);
  if (dtype_is_f32) {
    FEAT(float, 8, 2) FEAT(float, 16, 2) FEAT(float, 16, 4) FEAT(float, 24, 4) FEAT(float, 32, 4)
  } else {
    FEAT(double, 8, 2) FEAT(double, 16, 2) FEAT(double, 16, 4) FEAT(double, 24, 4) FEAT(double, 32, 4)
  }
#undef FEAT
  return hipErrorNotSupported;
}

hipError_t launch_lowmodes(int dtype_is_f32, const void* fhat, int rows, int half, int npair, int K, int Kh, int mh,
                           double box3, void* X, int ldx, float* rho, const double* mom, double L, int64_t cells,
                           void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dtype_is_f32)
    hipLaunchKernelGGL(k_lowmodes<float>, dim3(unsigned(cells)), dim3(256), 0, st, static_cast<const float*>(fhat),
                       rows, half, npair, K, Kh, mh, box3, static_cast<__bf16*>(X), ldx, rho, mom, L);
  else
    hipLaunchKernelGGL(k_lowmodes<double>, dim3(unsigned(cells)), dim3(256), 0, st,
                       static_cast<const double*>(fhat), rows, half, npair, K, Kh, mh, box3, static_cast<__bf16*>(X),
                       ldx, rho, mom, L);
  return hipGetLastError();
}

hipError_t launch_sur_output(const float* Y, int ldy, const float* rho, float scale, int n, double L, float* q,
                             double* r, int absolute, int64_t cells, void* stream) {
  hipLaunchKernelGGL(k_sur_output, dim3(unsigned(cells)), dim3(256), 0, static_cast<hipStream_t>(stream), Y, ldy, rho,
                     scale, n, L, q, r, absolute);
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

template <int N>
static hipError_t launch_shift_n(const float* in, int64_t ld_in, float* out, const double* mom, int sign, double L,
                                 const float* rho, float scale, int mode, double* r, int absolute, int64_t cells,
                                 hipStream_t st) {
  static bool attr_set = false;
  constexpr size_t lds = ShiftLds<N>::bytes;
  if (!attr_set) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_shift<N>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((k_shift<N>), dim3(unsigned(cells)), dim3(ShiftLds<N>::TPB), lds, st, in, ld_in, out, mom, sign,
                     L, rho, scale, mode, r, absolute);
  return hipGetLastError();
}

hipError_t launch_shift(int n, const float* in, int64_t ld_in, float* out, const double* mom, int sign, double L,
                        const float* rho, float scale, int mode, double* r, int absolute, int64_t cells,
                        void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (n) {
    case 8: return launch_shift_n<8>(in, ld_in, out, mom, sign, L, rho, scale, mode, r, absolute, cells, st);
    case 16: return launch_shift_n<16>(in, ld_in, out, mom, sign, L, rho, scale, mode, r, absolute, cells, st);
    case 24: return launch_shift_n<24>(in, ld_in, out, mom, sign, L, rho, scale, mode, r, absolute, cells, st);
    case 32: return launch_shift_n<32>(in, ld_in, out, mom, sign, L, rho, scale, mode, r, absolute, cells, st);
    default: return hipErrorInvalidValue;
  }
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
