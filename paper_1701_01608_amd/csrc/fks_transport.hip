// Exact-shift transport of the Fast Kinetic Scheme (Section 2.1 transport step,
// Section 3 particle interpretation with one generic cell).
//
// Built without fast-math and with FP contraction off: the integer shift of every
// velocity is decided by floor() of an FP64 expression whose operations and rounding
// order are part of the definition:
//   t = s + v*dt;  delta = floor((t + dx/2) / dx);  s = t - delta*dx;  o += delta.
#include <hip/hip_runtime.h>

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
  const int64_t cells = int64_t(nx) * ny * nz;
  const int64_t stride = gridDim.x / blocks_per_cell;
  for (int64_t cell = blockIdx.x / blocks_per_cell; cell < cells; cell += stride) {
    const int cx = int(cell / (int64_t(ny) * nz)), cy = int((cell / nz) % ny), cz = int(cell % nz);
    int sx = (cx - dx) % nx;
    int sy = (cy - dy) % ny;
    int sz = (cz - dz) % nz;
    sx += (sx < 0) ? nx : 0;
    sy += (sy < 0) ? ny : 0;
    sz += (sz < 0) ? nz : 0;
    const size_t src = (size_t(sx) * ny + sy) * nz + sz;
    fout[size_t(cell) * nv + k] = fin[src * nv + k];
  }
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

}  // namespace fks
