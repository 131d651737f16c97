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

// ------------------------------------------------------------------------------------
// Per-cell transport with the macroscopic variables (Section 3 eq. DM_update, Section 4.1
// sequential algorithm) and, optionally, the BGK relaxation (Section 2.2.1).
//
// One workgroup owns one destination cell j at a time (grid-stride over the cells):
//   1. DM_update: for every velocity k that moved this step (delta_k != 0) the sister
//      particle from cell j - delta_k replaces the particle that left, so
//      U_j += sum_k (f[j - delta_k][k] - f[j][k]) phi(v_k) dv^3 (FP64, fixed summation
//      order: bitwise reproducible); ToPrimitive gives (rho, u, T) from U_j.
//   2. the shifted masses f*[j][k] = f[j - delta_k][k] are written, or, with BGK, relaxed
//      at frozen U_j towards E_jk = M_jk (1 + lambda . phi(v_k)), the sampled Maxwellian
//      M = rho (2 pi T)^{-3/2} exp(-|v - u|^2 / 2T) times the affine factor in the
//      invariants that makes the discrete moments of E exactly U_j (so the relaxation
//      conserves what DM_update assumes it conserves): Euler f* + dt nu (E - f*) (eq.
//      disc_relax) or exact E + (f* - E) exp(-nu dt).  M is separable: one Gaussian factor
//      per axis in LDS, and every moment of M against two invariants is a product of three
//      1-D moments, which gives the 5 x 5 system for lambda per cell.
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

template <typename T, bool DM, int MODE>
__global__ __launch_bounds__(256) void k_step_cell(const T* __restrict__ fin, T* __restrict__ fout,
                                                   const int32_t* __restrict__ dl, StepCellArgs a) {
#pragma clang fp contract(off)
  constexpr int kMaxN = 64;
  __shared__ double red[5 * 16];
  __shared__ double sW[8];
  __shared__ double gd[3][kMaxN];
  __shared__ double sA[3][5];
  __shared__ double sLam[5];
  const int n = a.n, nv = n * n * n;
  const double dv = 2.0 * a.L / n, w3 = dv * dv * dv;
  const int64_t cells = int64_t(a.nx) * a.ny * a.nz;
  const int tid = threadIdx.x;
  T* q = static_cast<T*>(a.q);
  for (int64_t cell = blockIdx.x; cell < cells; cell += gridDim.x) {
    const int cx = int(cell / (int64_t(a.ny) * a.nz)), cy = int((cell / a.nz) % a.ny), cz = int(cell % a.nz);
    const T* fdst_old = fin + size_t(cell) * nv;
    auto source = [&](int k) {
      int sx = (cx - dl[3 * k + 0]) % a.nx, sy = (cy - dl[3 * k + 1]) % a.ny, sz = (cz - dl[3 * k + 2]) % a.nz;
      sx += (sx < 0) ? a.nx : 0;
      sy += (sy < 0) ? a.ny : 0;
      sz += (sz < 0) ? a.nz : 0;
      return ((size_t(sx) * a.ny + sy) * a.nz + sz) * size_t(nv) + size_t(k);
    };
    if constexpr (DM) {
      double acc[5] = {0, 0, 0, 0, 0};
      for (int k = tid; k < nv; k += blockDim.x) {
        if ((dl[3 * k + 0] | dl[3 * k + 1] | dl[3 * k + 2]) == 0) continue;
        const double diff = double(fin[source(k)]) - double(fdst_old[k]);
        const double vx = -a.L + double(k / (n * n)) * dv, vy = -a.L + double((k / n) % n) * dv,
                     vz = -a.L + double(k % n) * dv;
        acc[0] += diff;
        acc[1] += diff * vx;
        acc[2] += diff * vy;
        acc[3] += diff * vz;
        acc[4] += diff * (0.5 * (vx * vx + vy * vy + vz * vz));
      }
      block_sum5(acc, red);
      if (tid == 0) {
        double U[5], W[5];
        for (int i = 0; i < 5; ++i) {
          U[i] = a.cons[cell * 5 + i] + acc[i] * w3;
          a.cons[cell * 5 + i] = U[i];
        }
        to_primitive(U, W);
        if (a.prim)
          for (int i = 0; i < 5; ++i) a.prim[cell * 5 + i] = W[i];
        for (int i = 0; i < 5; ++i) sW[i] = W[i];
      }
      __syncthreads();
    }
    if constexpr (MODE != 0) {
      // the cell's Maxwellian: one Gaussian factor per axis
      const double T0 = sW[4];
      if (tid < 3 * n) {
        const int ax = tid / n, i = tid % n;
        const double d = -a.L + double(i) * dv - sW[1 + ax];
        gd[ax][i] = exp(-d * d / (2.0 * T0));
      }
      __syncthreads();
      // 1-D moments A[ax][p] = sum_i g_ax(v_i) v_i^p, p <= 4: every grid moment of the
      // separable M against a product of two invariants is a product of three of them
      if (tid < 15) {
        const int ax = tid / 5, pw = tid % 5;
        double acc = 0.0;
        for (int i = 0; i < n; ++i) {
          const double v = -a.L + double(i) * dv;
          double m = gd[ax][i];
          for (int e = 0; e < pw; ++e) m *= v;
          acc += m;
        }
        sA[ax][pw] = acc;
      }
      __syncthreads();
      if (tid == 0) {
        const double rho = sW[0];
        const double nu = a.nu_density ? a.nu * rho : a.nu;
        const double pref = rho * pow(2.0 * 3.14159265358979323846 * T0, -1.5);
        // invariants as polynomials: (coefficient, exponents of v_x, v_y, v_z)
        struct Term {
          double c;
          int p[3];
        };
        const Term terms[7] = {{1.0, {0, 0, 0}}, {1.0, {1, 0, 0}}, {1.0, {0, 1, 0}}, {1.0, {0, 0, 1}},
                               {0.5, {2, 0, 0}}, {0.5, {0, 2, 0}}, {0.5, {0, 0, 2}}};
        const int first[6] = {0, 1, 2, 3, 4, 7};  // phi_i = terms[first[i] .. first[i+1])
        auto mono = [&](const int* p, const int* q) {
          return sA[0][p[0] + q[0]] * sA[1][p[1] + q[1]] * sA[2][p[2] + q[2]];
        };
        const int zero[3] = {0, 0, 0};
        // G lambda = U / (pref dv^3) - m:  G_ij = sum_k g phi_i phi_j,  m_i = sum_k g phi_i
        double G[5][6];
        for (int i = 0; i < 5; ++i) {
          for (int j = 0; j < 5; ++j) {
            double acc = 0.0;
            for (int u = first[i]; u < first[i + 1]; ++u)
              for (int v = first[j]; v < first[j + 1]; ++v) acc += terms[u].c * terms[v].c * mono(terms[u].p, terms[v].p);
            G[i][j] = acc;
          }
          double m = 0.0;
          for (int u = first[i]; u < first[i + 1]; ++u) m += terms[u].c * mono(terms[u].p, zero);
          G[i][5] = a.cons[cell * 5 + i] / (pref * w3) - m;
        }
        for (int c = 0; c < 5; ++c) {  // Gauss-Jordan, partial pivoting
          int piv = c;
          for (int r = c + 1; r < 5; ++r)
            if (fabs(G[r][c]) > fabs(G[piv][c])) piv = r;
          if (piv != c)
            for (int k = 0; k < 6; ++k) {
              const double t = G[c][k];
              G[c][k] = G[piv][k];
              G[piv][k] = t;
            }
          const double inv = 1.0 / G[c][c];
          for (int k = c; k < 6; ++k) G[c][k] *= inv;
          for (int r = 0; r < 5; ++r)
            if (r != c) {
              const double fct = G[r][c];
              for (int k = c; k < 6; ++k) G[r][k] -= fct * G[c][k];
            }
        }
        for (int i = 0; i < 5; ++i) sLam[i] = G[i][5];
        sW[5] = pref;
        sW[6] = nu;
        sW[7] = MODE == 2 ? exp(-nu * a.dt) : nu * a.dt;
      }
      __syncthreads();
    }
    double mom[5] = {0, 0, 0, 0, 0};
    const double pref = MODE != 0 ? sW[5] : 0.0, nu_c = MODE != 0 ? sW[6] : 0.0, rate = MODE != 0 ? sW[7] : 0.0;
    for (int k = tid; k < nv; k += blockDim.x) {
      const T fs = fin[source(k)];
      T out = fs;
      const int ix = k / (n * n), iy = (k / n) % n, iz = k % n;
      if constexpr (MODE != 0) {
        const double vx = -a.L + double(ix) * dv, vy = -a.L + double(iy) * dv, vz = -a.L + double(iz) * dv;
        const double corr = 1.0 + sLam[0] + sLam[1] * vx + sLam[2] * vy + sLam[3] * vz +
                            sLam[4] * (0.5 * (vx * vx + vy * vy + vz * vz));
        const double E = pref * gd[0][ix] * gd[1][iy] * gd[2][iz] * corr;
        const double x = double(fs);
        if (q) q[size_t(cell) * nv + k] = T(nu_c * (E - x));
        out = T(MODE == 2 ? E + (x - E) * rate : x + rate * (E - x));
      }
      fout[size_t(cell) * nv + k] = out;
      if (a.moments) {
        const double d = double(out);
        const double vx = -a.L + double(ix) * dv, vy = -a.L + double(iy) * dv, vz = -a.L + double(iz) * dv;
        mom[0] += d;
        mom[1] += d * vx;
        mom[2] += d * vy;
        mom[3] += d * vz;
        mom[4] += d * (0.5 * (vx * vx + vy * vy + vz * vz));
      }
    }
    if (a.moments) {
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
  if (a.n > 64 || 3 * a.n > 256) return hipErrorInvalidValue;
  const int64_t cells = int64_t(a.nx) * a.ny * a.nz;
  const dim3 grid(unsigned(cells < (int64_t(1) << 20) ? cells : (int64_t(1) << 20)));
  hipStream_t st = static_cast<hipStream_t>(stream);
  prof_mark(kProfRoll, true, st);
#define FKS_STEP_CELL(T, D, M)                                                                               \
  hipLaunchKernelGGL((k_step_cell<T, D, M>), grid, dim3(256), 0, st, static_cast<const T*>(fin), static_cast<T*>(fout), \
                     dl, a)
  if (dtype_is_f32) {
    if (dm) {
      if (mode == 0) FKS_STEP_CELL(float, true, 0);
      else if (mode == 1) FKS_STEP_CELL(float, true, 1);
      else FKS_STEP_CELL(float, true, 2);
    } else {
      FKS_STEP_CELL(float, false, 0);
    }
  } else {
    if (dm) {
      if (mode == 0) FKS_STEP_CELL(double, true, 0);
      else if (mode == 1) FKS_STEP_CELL(double, true, 1);
      else FKS_STEP_CELL(double, true, 2);
    } else {
      FKS_STEP_CELL(double, false, 0);
    }
  }
#undef FKS_STEP_CELL
  prof_mark(kProfRoll, false, st);
  return hipGetLastError();
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
