// Exact-shift transport of the Fast Kinetic Scheme (Section 2.1 transport step,
// Section 3 particle interpretation with one generic cell).
//
// Built without fast-math and with FP contraction off: the integer shift of every
// velocity is decided by floor() of an FP64 expression whose operations and rounding
// order are part of the definition:
//   t = s + v*dt;  delta = floor((t + dx/2) / dx);  s = t - delta*dx;  o += delta.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "fks_internal.hpp"

namespace fks {

__global__ void k_xport_reset(double* s, int32_t* o, int32_t* dl, int m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) {
    s[i] = 0.0;
    o[i] = 0;
    dl[i] = 0;
  }
}

__global__ void k_xport_advance(double* s, int32_t* o, int32_t* dl, int n, double L, double dt, double dx) {
#pragma clang fp contract(off)
  const int nv = n * n * n;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nv) return;
  const double dv = 2.0 * L / n;
  const int idx[3] = {k / (n * n), (k / n) % n, k % n};
  for (int a = 0; a < 3; ++a) {
    const double v = -L + double(idx[a]) * dv;
    const double prod = v * dt;
    const double t = s[3 * k + a] + prod;
    const double u = (t + 0.5 * dx) / dx;
    const double d = floor(u);
    s[3 * k + a] = t - d * dx;
    dl[3 * k + a] = int32_t(d);
    o[3 * k + a] += int32_t(d);
  }
}

// (c - d) mod m for a shift d of at most one box length, without a division; larger shifts
// take the remainder
__device__ __forceinline__ int wrap_sub(int c, int d, int m) {
  int s = c - d;
  if (s < 0 || s >= m) {
    s += (s < 0) ? m : -m;
    if (s < 0 || s >= m) s = ((s % m) + m) % m;
  }
  return s;
}

// f_out[cell][k] = f_in[(cell - delta_k) mod box][k]; one thread per (cell, velocity),
// consecutive threads on consecutive velocities of one destination cell.  The grid holds
// blocks_per_cell blocks for each of a bounded number of cells and strides over the rest
// (the threads of one launch stay below 2^32 for any box).
template <typename T>
__global__ __launch_bounds__(256) void k_roll(const T* __restrict__ fin, T* __restrict__ fout,
                                              const int32_t* __restrict__ dl, int nv, int nx, int ny, int nz,
                                              int blocks_per_cell) {
  const int k = (blockIdx.x % blocks_per_cell) * blockDim.x + threadIdx.x;
  if (k >= nv) return;
  const int dx = dl[3 * k + 0], dy = dl[3 * k + 1], dz = dl[3 * k + 2];
  // boxes hold at most 2^24 cells: 32-bit cell indices
  const int cells = nx * ny * nz, nyz = ny * nz;
  const int stride = int(gridDim.x) / blocks_per_cell;
  for (int cell = int(blockIdx.x) / blocks_per_cell; cell < cells; cell += stride) {
    const int cx = cell / nyz, cyz = cell - cx * nyz, cy = cyz / nz, cz = cyz - cy * nz;
    const int src = (wrap_sub(cx, dx, nx) * ny + wrap_sub(cy, dy, ny)) * nz + wrap_sub(cz, dz, nz);
    fout[size_t(cell) * nv + k] = fin[size_t(src) * nv + k];
  }
}

// ------------------------------------------------------------------------------------
// The macroscopic variables of the FKS step (Section 3 eq. DM_update, Section 4.1
// sequential algorithm) and the BGK relaxation (Section 2.2.1), in three kernels:
//   k_dm_update   one workgroup per cell j: for every velocity k that moved this step
//                 (delta_k != 0) the sister particle from cell j - delta_k replaces the one
//                 that left, U_j += sum_k (f[j - delta_k][k] - f[j][k]) phi(v_k) dv^3 (FP64,
//                 fixed summation order: bitwise reproducible); ToPrimitive (rho, u, T).
//   k_bgk_setup   one thread per cell: E_jk = M_jk (1 + lambda . phi(v_k)), the sampled
//                 Maxwellian M = rho (2 pi T)^{-3/2} exp(-|v - u|^2 / 2T) times the affine
//                 factor in the invariants that gives E exactly the discrete moments U_j (so
//                 the relaxation conserves what DM_update assumes it conserves).  M is
//                 separable (one Gaussian factor per axis) and every grid moment of M against
//                 two invariants is a product of three 1-D moments: the 5 x 5 system for
//                 lambda is assembled in closed form and solved by Cholesky (it is symmetric
//                 positive definite).  The factors and constants are parked at the start of
//                 the cell's output block, which only this cell's relaxation workgroup writes.
//   k_bgk_relax   one workgroup per cell: reads its parked constants, then streams
//                 f*[j][k] = f[j - delta_k][k] relaxed at frozen U_j: Euler f* + dt nu (E - f*)
//                 (eq. disc_relax) or exact E + (f* - E) exp(-nu dt).
// Splitting keeps each streaming kernel's registers small (the per-cell setup in FP64,
// inlined into the streaming loop, held 150+ registers and left 2-3 waves per SIMD).
__device__ __forceinline__ void block_sum5(double (&v)[5], double* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int i = 0; i < 5; ++i) {
    double x = v[i];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) red[i * 16 + wid] = x;
  }
  __syncthreads();
  for (int i = 0; i < 5; ++i) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[i * 16 + w];
    v[i] = s;
  }
  __syncthreads();
}

__device__ __forceinline__ void to_primitive(const double* U, double* W) {
  const double rho = U[0];
  const double ux = U[1] / rho, uy = U[2] / rho, uz = U[3] / rho;
  W[0] = rho;
  W[1] = ux;
  W[2] = uy;
  W[3] = uz;
  W[4] = (2.0 / 3.0) * (U[4] / rho - 0.5 * (ux * ux + uy * uy + uz * uz));
}


// velocities per thread and pass of the streaming loops: their loads are all issued
// before any is used, so that a wave keeps several gathers in flight; the pass loop itself
// is not unrolled
constexpr int kStreamUnroll = 8;
constexpr int kStreamThreads = 256;

// source element of velocity k for destination cell (cx, cy, cz)
__device__ __forceinline__ size_t source_index(int cx, int cy, int cz, int dx, int dy, int dz, int nx, int ny,
                                               int nz, int nv, int k) {
  return ((size_t(wrap_sub(cx, dx, nx)) * ny + wrap_sub(cy, dy, ny)) * nz + wrap_sub(cz, dz, nz)) * size_t(nv) +
         size_t(k);
}

template <typename T, int N>
__global__ __launch_bounds__(256) void k_dm_update(const T* __restrict__ fin, const int32_t* __restrict__ dl,
                                                   StepCellArgs a) {
#pragma clang fp contract(off)
  constexpr int nv = N * N * N, UNR = kStreamUnroll, NTH = kStreamThreads;
  __shared__ double red[5 * 16];
  const double dv = 2.0 * a.L / N, w3 = dv * dv * dv;
  const int64_t cells = int64_t(a.nx) * a.ny * a.nz;
  const int tid = threadIdx.x;
  for (int64_t cell = blockIdx.x; cell < cells; cell += gridDim.x) {
    const int cx = int(cell / (int64_t(a.ny) * a.nz)), cy = int((cell / a.nz) % a.ny), cz = int(cell % a.nz);
    const T* fold = fin + size_t(cell) * nv;
    double acc[5] = {0, 0, 0, 0, 0};
#pragma unroll 1
    for (int k0 = 0; k0 < nv; k0 += NTH * UNR) {
      T va[UNR], vb[UNR];
      bool mv[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int k = k0 + u * NTH + tid;
        mv[u] = false;
        va[u] = vb[u] = T(0);
        if (k < nv) {
          const int dx = dl[3 * k + 0], dy = dl[3 * k + 1], dz = dl[3 * k + 2];
          mv[u] = (dx | dy | dz) != 0;
          if (mv[u]) {
            va[u] = fin[source_index(cx, cy, cz, dx, dy, dz, a.nx, a.ny, a.nz, nv, k)];
            vb[u] = fold[k];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        if (!mv[u]) continue;
        const int k = k0 + u * NTH + tid;
        const double diff = double(va[u]) - double(vb[u]);
        const double vx = -a.L + double(k / (N * N)) * dv, vy = -a.L + double((k / N) % N) * dv,
                     vz = -a.L + double(k % N) * dv;
        acc[0] += diff;
        acc[1] += diff * vx;
        acc[2] += diff * vy;
        acc[3] += diff * vz;
        acc[4] += diff * (0.5 * (vx * vx + vy * vy + vz * vz));
      }
    }
    block_sum5(acc, red);
    if (tid == 0) {
      double U[5], W[5];
      for (int i = 0; i < 5; ++i) {
        U[i] = a.cons[cell * 5 + i] + acc[i] * w3;
        a.cons[cell * 5 + i] = U[i];
      }
      if (a.prim) {
        to_primitive(U, W);
        for (int i = 0; i < 5; ++i) a.prim[cell * 5 + i] = W[i];
      }
    }
  }
}

// parked per-cell constants of the relaxation, in doubles at the start of the cell's
// output block: [0] pref, [1] nu, [2] rate (exp(-nu dt) or nu dt), [3..7] lambda,
// [8 .. 8 + 3N) the Gaussian factors of the three axes
template <int N>
struct BgkPark {
  static constexpr int kDoubles = 8 + 3 * N;
};

template <typename T, int N, int MODE>
__global__ __launch_bounds__(256) void k_bgk_setup(T* __restrict__ fout, StepCellArgs a) {
  constexpr int nv = N * N * N;
  static_assert(size_t(BgkPark<N>::kDoubles) * sizeof(double) <= size_t(nv) * sizeof(T), "cell too small to park");
  const int64_t cells = int64_t(a.nx) * a.ny * a.nz;
  const int64_t cell = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (cell >= cells) return;
  const double dv = 2.0 * a.L / N, w3 = dv * dv * dv;
  double U[5], W[5];
  for (int i = 0; i < 5; ++i) U[i] = a.cons[cell * 5 + i];
  to_primitive(U, W);
  double* park = reinterpret_cast<double*>(fout + size_t(cell) * nv);
  // Gaussian factors and their 1-D moments A[ax][p] = sum_i g_ax(v_i) v_i^p, p <= 4
  double A[3][5];
  for (int ax = 0; ax < 3; ++ax) {
    for (int p = 0; p < 5; ++p) A[ax][p] = 0.0;
    for (int i = 0; i < N; ++i) {
      const double v = -a.L + double(i) * dv;
      const double d = v - W[1 + ax];
      const double g = exp(-d * d / (2.0 * W[4]));
      park[8 + ax * N + i] = g;
      A[ax][0] += g;
      A[ax][1] += g * v;
      A[ax][2] += g * v * v;
      A[ax][3] += g * v * v * v;
      A[ax][4] += g * v * v * v * v;
    }
  }
  auto m3 = [&](int px, int py, int pz) { return A[0][px] * A[1][py] * A[2][pz]; };
  // G_ij = sum_k g phi_i phi_j over phi = (1, v_x, v_y, v_z, |v|^2/2); m_i = G_0i
  double G[5][5];
  G[0][0] = m3(0, 0, 0);
  G[0][1] = m3(1, 0, 0);
  G[0][2] = m3(0, 1, 0);
  G[0][3] = m3(0, 0, 1);
  G[0][4] = 0.5 * (m3(2, 0, 0) + m3(0, 2, 0) + m3(0, 0, 2));
  G[1][1] = m3(2, 0, 0);
  G[1][2] = m3(1, 1, 0);
  G[1][3] = m3(1, 0, 1);
  G[1][4] = 0.5 * (m3(3, 0, 0) + m3(1, 2, 0) + m3(1, 0, 2));
  G[2][2] = m3(0, 2, 0);
  G[2][3] = m3(0, 1, 1);
  G[2][4] = 0.5 * (m3(2, 1, 0) + m3(0, 3, 0) + m3(0, 1, 2));
  G[3][3] = m3(0, 0, 2);
  G[3][4] = 0.5 * (m3(2, 0, 1) + m3(0, 2, 1) + m3(0, 0, 3));
  G[4][4] = 0.25 * (m3(4, 0, 0) + m3(0, 4, 0) + m3(0, 0, 4)) + 0.5 * (m3(2, 2, 0) + m3(2, 0, 2) + m3(0, 2, 2));
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < i; ++j) G[i][j] = G[j][i];
  const double tt = 2.0 * 3.14159265358979323846 * W[4];
  const double pref = W[0] / (tt * sqrt(tt));
  double lam[5];
  for (int i = 0; i < 5; ++i) lam[i] = U[i] / (pref * w3) - G[0][i];
  // G = C C^T (C lower, in place), then C y = b, C^T lambda = y
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    double d = G[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) d -= G[j][k] * G[j][k];
    G[j][j] = sqrt(d);
    const double inv = 1.0 / G[j][j];
#pragma unroll
    for (int i = j + 1; i < 5; ++i) {
      double v = G[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= G[i][k] * G[j][k];
      G[i][j] = v * inv;
    }
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    double v = lam[i];
#pragma unroll
    for (int k = 0; k < i; ++k) v -= G[i][k] * lam[k];
    lam[i] = v / G[i][i];
  }
#pragma unroll
  for (int i = 4; i >= 0; --i) {
    double v = lam[i];
#pragma unroll
    for (int k = i + 1; k < 5; ++k) v -= G[k][i] * lam[k];
    lam[i] = v / G[i][i];
  }
  const double nu = a.nu_density ? a.nu * W[0] : a.nu;
  park[0] = pref;
  park[1] = nu;
  park[2] = MODE == 2 ? exp(-nu * a.dt) : nu * a.dt;
  for (int i = 0; i < 5; ++i) park[3 + i] = lam[i];
}

// EXTRAS: the collision operator and/or the direct moments are also written (last step);
// without them the streaming loop holds no FP64 accumulators
template <typename T, int N, int MODE, bool EXTRAS>
__global__ __launch_bounds__(256) void k_bgk_relax(const T* __restrict__ fin, T* __restrict__ fout,
                                                   const int32_t* __restrict__ dl, StepCellArgs a) {
#pragma clang fp contract(off)
  constexpr int nv = N * N * N, UNR = kStreamUnroll, NTH = kStreamThreads, NP = BgkPark<N>::kDoubles;
  // the Maxwellian and the relaxation are evaluated in the storage precision (FP32 cells:
  // a few FP32 roundings, far below the rounding of the stored result's neighbours; FP64:
  // FP64); the optional moments are FP64 sums
  using R = T;
  __shared__ double red[5 * 16];
  __shared__ R sp[NP];
  const double dv = 2.0 * a.L / N, w3 = dv * dv * dv;
  const R Lr = R(a.L), dvr = R(dv);
  const int64_t cells = int64_t(a.nx) * a.ny * a.nz;
  const int tid = threadIdx.x;
  T* q = static_cast<T*>(a.q);
  for (int64_t cell = blockIdx.x; cell < cells; cell += gridDim.x) {
    const int cx = int(cell / (int64_t(a.ny) * a.nz)), cy = int((cell / a.nz) % a.ny), cz = int(cell % a.nz);
    T* fo = fout + size_t(cell) * nv;
    if (tid < NP) sp[tid] = R(reinterpret_cast<const double*>(fo)[tid]);
    __syncthreads();  // the parked constants are read before the cell's block is overwritten
    const R pref = sp[0], nu_c = sp[1], rate = sp[2];
    double mom[5] = {0, 0, 0, 0, 0};
#pragma unroll 1
    for (int k0 = 0; k0 < nv; k0 += NTH * UNR) {
      T vs[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int k = k0 + u * NTH + tid;
        vs[u] = T(0);
        if (k < nv)
          vs[u] = fin[source_index(cx, cy, cz, dl[3 * k + 0], dl[3 * k + 1], dl[3 * k + 2], a.nx, a.ny, a.nz, nv, k)];
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int k = k0 + u * NTH + tid;
        if (k >= nv) continue;
        const int ix = k / (N * N), iy = (k / N) % N, iz = k % N;
        const R vx = -Lr + R(ix) * dvr, vy = -Lr + R(iy) * dvr, vz = -Lr + R(iz) * dvr;
        const R corr = R(1) + sp[3] + sp[4] * vx + sp[5] * vy + sp[6] * vz +
                       sp[7] * (R(0.5) * (vx * vx + vy * vy + vz * vz));
        const R E = pref * sp[8 + ix] * sp[8 + N + iy] * sp[8 + 2 * N + iz] * corr;
        const R x = vs[u];
        const T out = MODE == 2 ? E + (x - E) * rate : x + rate * (E - x);
        fo[k] = out;
        if constexpr (EXTRAS) {
          if (q) q[size_t(cell) * nv + k] = nu_c * (E - x);
        }
        if (EXTRAS && a.moments) {
          const double d = double(out);
          const double wx = -a.L + double(ix) * dv, wy = -a.L + double(iy) * dv, wz = -a.L + double(iz) * dv;
          mom[0] += d;
          mom[1] += d * wx;
          mom[2] += d * wy;
          mom[3] += d * wz;
          mom[4] += d * (0.5 * (wx * wx + wy * wy + wz * wz));
        }
      }
    }
    if (EXTRAS && a.moments) {
      block_sum5(mom, red);
      if (tid == 0)
        for (int i = 0; i < 5; ++i) a.moments[cell * 5 + i] = mom[i] * w3;
    }
    __syncthreads();  // LDS of this cell is reused by the next one
  }
}

// ToPrimitive of [cells][5] conservative variables (in may equal out)
__global__ void k_to_primitive(const double* in, double* out, int64_t cells) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= cells) return;
  double U[5], W[5];
  for (int i = 0; i < 5; ++i) U[i] = in[c * 5 + i];
  to_primitive(U, W);
  for (int i = 0; i < 5; ++i) out[c * 5 + i] = W[i];
}

template <typename T>
__global__ __launch_bounds__(256) void k_copy(const T* __restrict__ src, T* __restrict__ dst, int64_t n) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

hipError_t launch_xport_reset(const XportState& st, int nv, void* stream) {
  const int m = 3 * nv;
  hipLaunchKernelGGL(k_xport_reset, dim3((m + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream), st.s,
                     st.o, st.dl, m);
  return hipGetLastError();
}

hipError_t launch_xport_advance(const XportState& st, int n, double L, double dt, double dx, void* stream) {
  const int nv = n * n * n;
  prof_mark(kProfAdvance, true, static_cast<hipStream_t>(stream));
  hipLaunchKernelGGL(k_xport_advance, dim3((nv + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream),
                     st.s, st.o, st.dl, n, L, dt, dx);
  prof_mark(kProfAdvance, false, static_cast<hipStream_t>(stream));
  return hipGetLastError();
}

hipError_t launch_roll(int dtype_is_f32, const void* fin, void* fout, const int32_t* dl, int nv, int nx, int ny,
                       int nz, void* stream) {
  const int bpc = (nv + 255) / 256;
  const long cells = long(nx) * ny * nz;
  // at most 2^22 blocks (2^30 threads); each block strides over its cells
  const long max_cells = (1L << 22) / bpc > 0 ? (1L << 22) / bpc : 1;
  const dim3 grid(unsigned((cells < max_cells ? cells : max_cells) * bpc));
  hipStream_t st = static_cast<hipStream_t>(stream);
  prof_mark(kProfRoll, true, st);
  if (dtype_is_f32)
    hipLaunchKernelGGL(k_roll<float>, grid, dim3(256), 0, st, static_cast<const float*>(fin),
                       static_cast<float*>(fout), dl, nv, nx, ny, nz, bpc);
  else
    hipLaunchKernelGGL(k_roll<double>, grid, dim3(256), 0, st, static_cast<const double*>(fin),
                       static_cast<double*>(fout), dl, nv, nx, ny, nz, bpc);
  prof_mark(kProfRoll, false, st);
  return hipGetLastError();
}

hipError_t launch_step_cell(int dtype_is_f32, const void* fin, void* fout, const int32_t* dl, int dm, int mode,
                            const StepCellArgs& a, void* stream) {
  const int64_t cells = int64_t(a.nx) * a.ny * a.nz;
  const dim3 grid(unsigned(cells < (int64_t(1) << 20) ? cells : (int64_t(1) << 20)));
  hipStream_t st = static_cast<hipStream_t>(stream);
  // the relaxation needs the DM-updated U; without a relaxation this is the DM update only
  if (!dm) return hipErrorInvalidValue;
  auto go = [&](auto tag, auto nc) -> hipError_t {
    using T = decltype(tag);
    constexpr int NN = decltype(nc)::value;
    const T* fi = static_cast<const T*>(fin);
    T* fo = static_cast<T*>(fout);
    hipLaunchKernelGGL((k_dm_update<T, NN>), grid, dim3(kStreamThreads), 0, st, fi, dl, a);
    if (mode == 0) return hipGetLastError();
    const dim3 sgrid(unsigned((cells + 255) / 256));
    const bool extras = a.q || a.moments;
    if (mode == 1) {
      hipLaunchKernelGGL((k_bgk_setup<T, NN, 1>), sgrid, dim3(256), 0, st, fo, a);
      if (extras) hipLaunchKernelGGL((k_bgk_relax<T, NN, 1, true>), grid, dim3(kStreamThreads), 0, st, fi, fo, dl, a);
      else hipLaunchKernelGGL((k_bgk_relax<T, NN, 1, false>), grid, dim3(kStreamThreads), 0, st, fi, fo, dl, a);
    } else {
      hipLaunchKernelGGL((k_bgk_setup<T, NN, 2>), sgrid, dim3(256), 0, st, fo, a);
      if (extras) hipLaunchKernelGGL((k_bgk_relax<T, NN, 2, true>), grid, dim3(kStreamThreads), 0, st, fi, fo, dl, a);
      else hipLaunchKernelGGL((k_bgk_relax<T, NN, 2, false>), grid, dim3(kStreamThreads), 0, st, fi, fo, dl, a);
    }
    return hipGetLastError();
  };
  auto by_n = [&](auto tag) -> hipError_t {
    switch (a.n) {
      case 8: return go(tag, std::integral_constant<int, 8>{});
      case 12: return go(tag, std::integral_constant<int, 12>{});
      case 16: return go(tag, std::integral_constant<int, 16>{});
      case 24: return go(tag, std::integral_constant<int, 24>{});
      case 32: return go(tag, std::integral_constant<int, 32>{});
      default: return hipErrorInvalidValue;
    }
  };
  prof_mark(kProfRoll, true, st);
  const hipError_t e = dtype_is_f32 ? by_n(float{}) : by_n(double{});
  prof_mark(kProfRoll, false, st);
  return e;
}

hipError_t launch_to_primitive(const double* in, double* out, int64_t cells, void* stream) {
  if (cells <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_primitive, dim3(unsigned((cells + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), in, out, cells);
  return hipGetLastError();
}

hipError_t launch_copy(int dtype_is_f32, const void* src, void* dst, int64_t n, void* stream) {
  const int64_t blocks = (n + 255) / 256;
  const dim3 grid(unsigned(blocks < (int64_t(1) << 22) ? (blocks > 0 ? blocks : 1) : (int64_t(1) << 22)));
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dtype_is_f32)
    hipLaunchKernelGGL(k_copy<float>, grid, dim3(256), 0, st, static_cast<const float*>(src), static_cast<float*>(dst), n);
  else
    hipLaunchKernelGGL(k_copy<double>, grid, dim3(256), 0, st, static_cast<const double*>(src),
                       static_cast<double*>(dst), n);
  return hipGetLastError();
}

}  // namespace fks
