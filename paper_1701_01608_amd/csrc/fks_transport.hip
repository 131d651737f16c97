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

__global__ void k_xport_reset(double* s, int32_t* o, int32_t* dl, int32_t* d1, int m, int m1) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) {
    s[i] = 0.0;
    o[i] = 0;
    dl[i] = 0;
  }
  if (i < m1) d1[i] = 0;
}

// The shift along axis a depends on the velocity's index along a only: every velocity
// with the same component has the same offset history.  Besides the per-velocity state,
// the velocities whose other two indices are zero add the step's shift of their axis to
// the compact table d1[a][i] of shifts pending since f was last moved; the streaming
// kernels apply the pending shifts and k_clear_pending then zeroes them (steps that only
// advance the offsets leave f in place and accumulate there).
__global__ void k_xport_advance(double* s, int32_t* o, int32_t* dl, int32_t* d1, int n, double L, double dt,
                                double dx) {
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
    if (idx[(a + 1) % 3] == 0 && idx[(a + 2) % 3] == 0) d1[a * n + idx[a]] += int32_t(d);
  }
}

__global__ void k_clear_pending(int32_t* d1, int m1) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m1) d1[i] = 0;
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

// ------------------------------------------------------------------------------------
// One transport step per cell, with the macroscopic variables of the FKS step (Section 3
// eq. DM_update, Section 4.1 sequential algorithm) and the BGK relaxation (Section 2.2.1),
// in one kernel: one workgroup per destination cell j, streaming the cell's shifted
// masses f*[j][k] = f[j - delta_k][k] in batches (for the relaxation after the per-cell
// setup, a cell of at most 64 KB reads them back from LDS, a larger one streams them a
// second time, mostly from L2).
//   MODE 3  shift only: f_out = f*.
//   MODE 0  shift and eq. DM_update: for every velocity k that moved this step
//           (delta_k != 0) the sister particle from cell j - delta_k replaces the one that
//           left, U_j += sum_k (f[j - delta_k][k] - f[j][k]) phi(v_k) dv^3 (FP64, fixed
//           summation order: bitwise reproducible); ToPrimitive (rho, u, T) when asked.
//   MODE 1  eq. DM_update, then the Euler relaxation f* + dt nu (E - f*) (eq. disc_relax),
//   MODE 2  or the exact one E + (f* - E) exp(-nu dt), at the frozen updated U_j.
// E_jk = M_jk (1 + lambda . phi(v_k)): the sampled Maxwellian M = rho (2 pi T)^{-3/2}
// exp(-|v - u|^2 / 2T) of the updated U_j times the affine factor in the invariants that
// gives E exactly the discrete moments U_j, so the relaxation conserves what DM_update
// assumes it conserves.  M is separable (one Gaussian factor per axis) and every grid
// moment of M against two invariants is a product of three 1-D moments: the 5 x 5 system
// for lambda is assembled in closed form and solved by Cholesky (it is symmetric positive
// definite).  Its setup runs once per cell between the two passes, each step spread over
// threads through LDS.
//
// The shift of axis a depends on the velocity index along a only (the compact table d1),
// so the source cell of velocity k is (sx[ix], sy[iy], sz[iz]) from three per-cell
// tables.  Consecutive lanes take consecutive velocities of the destination cell, so
// every load reads runs of consecutive values of one source cell and every store is
// contiguous.  Workgroups are dealt to the 8 XCDs round-robin; each XCD gets a contiguous
// range of cells, so the z neighbours a cell reads from, and the own-cell values of the
// moved velocities that a z neighbour reads as its shifted masses, meet in one L2.
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

// threads per cell: velocity k = u NTH + t of thread t (u < VPT), so lanes take
// consecutive velocities.  The workgroup is either m whole (v_y, v_z) planes (H = 1:
// m N^2 threads, m | N, a multiple of 64), where a thread's y and z indices are fixed, or
// half a plane (H = 2: N^2 / 2 threads, n = 32), where its y index alternates between two
// values with the parity of u; ix = (u / H) m + t / N^2.  Half planes at n = 32 keep two
// workgroups per CU, so one cell's setup overlaps another cell's streaming.
template <typename T, int N>
struct CellShape {
  static constexpr int NV = N * N * N;
  static constexpr int H = N >= 32 ? 2 : 1;
  static constexpr int M = H == 2 ? 1 : ((N * N) % 64 == 0 ? (N * N >= 256 ? 1 : 256 / (N * N)) : 4);
  static constexpr int NTH = M * N * N / H;
  static constexpr int VPT = NV / NTH;
  static constexpr int YH = N / H;   // y indices per half
  // values per streaming batch: the largest divisor of VPT up to 16 (n = 32) or 8 (smaller
  // workgroups, where more of them share a CU)
  static constexpr int batch() {
    for (int b = N >= 32 ? 16 : 8; b > 1; --b)
      if (VPT % b == 0 && b % H == 0) return b;
    return 1;
  }
  static constexpr int B = batch();
  // waves per SIMD the register allocation must allow: small cells are latency bound and
  // need many workgroups per CU in flight
  static constexpr int MIN_WAVES = N >= 32 ? 4 : 1;
  static_assert(N % M == 0 && NTH % 64 == 0 && NTH <= 1024 && NV % NTH == 0, "workgroup shape");
};

// Entry (i, j) of the Gram matrix G_ij = sum_k g(v_k) phi_i phi_j of the separable
// Gaussian g over phi = (1, v_x, v_y, v_z, |v|^2/2), from the 1-D moments
// A[ax][p] = sum_i g_ax(v_i) v_i^p (p <= 4): each grid moment of a monomial is a product of
// three 1-D moments.  i <= j.
__device__ __forceinline__ double gram_entry(int i, int j, const double (*A)[5]) {
  auto m3 = [&](int px, int py, int pz) { return A[0][px] * A[1][py] * A[2][pz]; };
  switch (i * 5 + j) {
    case 0: return m3(0, 0, 0);
    case 1: return m3(1, 0, 0);
    case 2: return m3(0, 1, 0);
    case 3: return m3(0, 0, 1);
    case 4: return 0.5 * (m3(2, 0, 0) + m3(0, 2, 0) + m3(0, 0, 2));
    case 6: return m3(2, 0, 0);
    case 7: return m3(1, 1, 0);
    case 8: return m3(1, 0, 1);
    case 9: return 0.5 * (m3(3, 0, 0) + m3(1, 2, 0) + m3(1, 0, 2));
    case 12: return m3(0, 2, 0);
    case 13: return m3(0, 1, 1);
    case 14: return 0.5 * (m3(2, 1, 0) + m3(0, 3, 0) + m3(0, 1, 2));
    case 18: return m3(0, 0, 2);
    case 19: return 0.5 * (m3(2, 0, 1) + m3(0, 2, 1) + m3(0, 0, 3));
    default:  // (4, 4)
      return 0.25 * (m3(4, 0, 0) + m3(0, 4, 0) + m3(0, 0, 4)) + 0.5 * (m3(2, 2, 0) + m3(2, 0, 2) + m3(0, 2, 2));
  }
}

// Solves G lambda = b for the symmetric positive definite 5 x 5 G (upper triangle given)
// by Cholesky, G = C C^T: C y = b, C^T lambda = y.  One thread, unrolled (in registers).
__device__ __forceinline__ void solve5(const double (*G)[5], double* b) {
  double C[5][5];
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    double d = G[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) d -= C[j][k] * C[j][k];
    C[j][j] = sqrt(d);
    const double inv = 1.0 / C[j][j];
#pragma unroll
    for (int i = j + 1; i < 5; ++i) {
      double v = G[j][i];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= C[i][k] * C[j][k];
      C[i][j] = v * inv;
    }
  }
  double y[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    double v = b[i];
#pragma unroll
    for (int k = 0; k < i; ++k) v -= C[i][k] * y[k];
    y[i] = v / C[i][i];
  }
#pragma unroll
  for (int i = 4; i >= 0; --i) {
    double v = y[i];
#pragma unroll
    for (int k = i + 1; k < 5; ++k) v -= C[k][i] * b[k];
    b[i] = v / C[i][i];
  }
}

// EXTRAS (BGK modes): the collision operator nu (E - f*) and/or the direct moments of the
// output are also written (last step); without them the streaming loop holds no FP64
// accumulators
template <typename T, int N, int MODE, bool EXTRAS>
__global__ __launch_bounds__((CellShape<T, N>::NTH), (CellShape<T, N>::MIN_WAVES)) void k_cell_step(const T* __restrict__ fin,
                                                                    T* __restrict__ fout,
                                                                    const int32_t* __restrict__ d1,
                                                                    StepCellArgs a) {
#pragma clang fp contract(off)
  using CS = CellShape<T, N>;
  constexpr int NV = CS::NV, NTH = CS::NTH, VPT = CS::VPT;
  constexpr bool DM = MODE != 3, BGK = MODE == 1 || MODE == 2;
  // cells of at most 64 KB keep their shifted masses in LDS between the two passes (each
  // thread reads back what it wrote); larger ones stream them a second time from the caches
  constexpr bool STAGE = BGK && CS::NV * sizeof(T) <= 64 * 1024;
  extern __shared__ __align__(16) unsigned char stage_raw[];
  T* stage = reinterpret_cast<T*>(stage_raw);
  // the Maxwellian and the relaxation are evaluated in the storage precision (FP32 cells:
  // a few FP32 roundings, far below the rounding of the stored result's neighbours; FP64:
  // FP64); the sums of DM_update and the optional moments are FP64
  using R = T;
  __shared__ int src_ax[3][N];   // wrapped source coordinate per axis index
  __shared__ double red[5 * 16];
  __shared__ double Ush[5], Wsh[5], par[8];
  __shared__ double gpow[3][5][N];
  __shared__ double Ash[3][5], Gsh[5][5];
  __shared__ R gr[3 * N];
  const double dv = 2.0 * a.L / N, w3 = dv * dv * dv;
  const int cells = a.nx * a.ny * a.nz, nyz = a.ny * a.nz;
  const int tid = threadIdx.x;
  T* q = static_cast<T*>(a.q);
  // rounds of gridDim.x cells; within a round XCD x (blockIdx % 8) takes a contiguous range
  const int per_xcd = int(gridDim.x) >> 3;
  const int slot = int(blockIdx.x & 7) * per_xcd + int(blockIdx.x >> 3);
  for (int base = 0; base < cells; base += int(gridDim.x)) {
    const int cell = base + slot;
    if (cell >= cells) break;  // uniform over the workgroup
    const int cx = cell / nyz, cyz = cell - cx * nyz, cy = cyz / a.nz, cz = cyz - cy * a.nz;
    if (tid < 3 * N) {
      const int ax = tid / N, i = tid - ax * N;
      const int d = d1[ax * N + i];
      const int c = ax == 0 ? cx : (ax == 1 ? cy : cz), m = ax == 0 ? a.nx : (ax == 1 ? a.ny : a.nz);
      src_ax[ax][i] = wrap_sub(c, d, m);
    }
    __syncthreads();
    const T* fown = fin + size_t(cell) * NV;
    T* fo = fout + size_t(cell) * NV;
    constexpr int MM = CS::M, H = CS::H, YH = CS::YH;
    // an opaque copy of the thread index per cell: the per-velocity offsets and abscissae
    // below are formed where they are used instead of being hoisted out of the cell loop
    int tcell = tid;
    asm volatile("" : "+v"(tcell));
    const int ix0 = tcell / (N * N), iy0 = (tcell / N) % YH, iz = tcell % N;
    // velocity k of this cell comes from the source cell (sx[ix], sy[iy], sz[iz]), element
    // (sx nyz + row(iy, iz)) NV + k.  With m = 1 the x index of value u is the same over
    // the workgroup, so the source plane sx nyz NV is a scalar base and the rest a 32-bit
    // offset (a y-z plane of the box holds fewer than 2^31 values)
    int row[H];
#pragma unroll
    for (int h = 0; h < H; ++h) row[h] = src_ax[1][iy0 + h * YH] * a.nz + src_ax[2][iz];
    auto load_shifted = [&](int u) -> T {
      if constexpr (MM == 1) {
        const int sx = __builtin_amdgcn_readfirstlane(src_ax[0][u / H]);
        const T* plane = fin + size_t(sx) * size_t(nyz) * NV;
        return plane[uint32_t(row[u % H]) * NV + uint32_t(u * NTH + tcell)];
      } else {
        return fin[(size_t(src_ax[0][(u / H) * MM + ix0]) * nyz + size_t(row[u % H])) * NV + size_t(u * NTH + tcell)];
      }
    };
    // The values stream in batches of B (the loads of a batch are all issued before any is
    // used); after the per-cell setup the relaxation reads the shifted masses back from LDS
    // (STAGE) or streams them a second time from the caches, instead of holding them in
    // registers across the setup.
    constexpr int B = CS::B;
    const double vz = -a.L + double(iz) * dv;
    // eq. DM_update: the sister particle of every moved velocity.  The own-cell value is
    // read for every velocity: for one that did not move it is the value just loaded as f*
    // (same address: a cache hit) and its difference is exactly zero, which leaves the
    // FP64 sums unchanged, so no branch holds the loads back.  Per y half the thread's y
    // and z abscissae are fixed, so the five moments of the differences follow from three
    // sums with the exact integer weights ix, ix^2 (v_x = -L + ix dv):
    // sum d v_x = -L D0 + dv D1, sum d v_x^2 = L^2 D0 - 2 L dv D1 + dv^2 D2
    double d0[H], d1s[H], d2[H];
#pragma unroll
    for (int h = 0; h < H; ++h) d0[h] = d1s[h] = d2[h] = 0.0;
#pragma unroll 1
    for (int u0 = 0; u0 < VPT; u0 += B) {
      T xs[B], vo[B];
#pragma unroll
      for (int j = 0; j < B; ++j) {
        xs[j] = load_shifted(u0 + j);
        if constexpr (DM) vo[j] = fown[uint32_t((u0 + j) * NTH + tcell)];
      }
      if constexpr (STAGE) {
#pragma unroll
        for (int j = 0; j < B; ++j) stage[(u0 + j) * NTH + tcell] = xs[j];
      }
      if constexpr (!BGK) {
#pragma unroll
        for (int j = 0; j < B; ++j) fo[uint32_t((u0 + j) * NTH + tcell)] = xs[j];
      }
      if constexpr (DM) {
#pragma unroll
        for (int j = 0; j < B; ++j) {
          const int h = j % H;   // B is a multiple of H
          const double diff = double(xs[j]) - double(vo[j]);
          const double ixd = double(((u0 + j) / H) * MM + ix0);
          d0[h] += diff;
          d1s[h] += diff * ixd;
          d2[h] += diff * (ixd * ixd);
        }
      }
    }
    if constexpr (DM) {
      double acc[5] = {0, 0, 0, 0, 0};
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const double vy = -a.L + double(iy0 + h * YH) * dv;
        const double sx1 = -a.L * d0[h] + dv * d1s[h];
        const double sx2 = a.L * a.L * d0[h] - 2.0 * a.L * dv * d1s[h] + dv * dv * d2[h];
        acc[0] += d0[h];
        acc[1] += sx1;
        acc[2] += vy * d0[h];
        acc[3] += vz * d0[h];
        acc[4] += 0.5 * (sx2 + (vy * vy + vz * vz) * d0[h]);
      }
      block_sum5(acc, red);
      if (tid == 0) {
        double U[5], W[5];
        for (int i = 0; i < 5; ++i) {
          U[i] = a.cons[size_t(cell) * 5 + i] + acc[i] * w3;
          a.cons[size_t(cell) * 5 + i] = U[i];
        }
        to_primitive(U, W);
        if (a.prim)
          for (int i = 0; i < 5; ++i) a.prim[size_t(cell) * 5 + i] = W[i];
        for (int i = 0; i < 5; ++i) {
          Ush[i] = U[i];
          Wsh[i] = W[i];
        }
      }
    }
    if constexpr (BGK) {
      // the cell's Maxwellian: Gaussian factors and their powers, the 1-D moments, the
      // Gram matrix and lambda, each step spread over threads through LDS
      __syncthreads();
      if (tid < 3 * N) {
        const int ax = tid / N, i = tid - ax * N;
        const double v = -a.L + double(i) * dv;
        const double d = v - Wsh[1 + ax];
        const double g = exp(-d * d / (2.0 * Wsh[4]));
        gr[tid] = R(g);
        double gp = g;
#pragma unroll
        for (int p = 0; p < 5; ++p) {
          gpow[ax][p][i] = gp;   // g v^p
          gp *= v;
        }
      }
      __syncthreads();
      if (tid < 15) {
        const int ax = tid / 5, p = tid - ax * 5;
        double m = 0.0;
#pragma unroll 1
        for (int i = 0; i < N; ++i) m += gpow[ax][p][i];
        Ash[ax][p] = m;
      }
      __syncthreads();
      if (tid < 25) {
        const int i = tid / 5, j = tid - i * 5;
        if (i <= j) Gsh[i][j] = gram_entry(i, j, Ash);
      }
      __syncthreads();
      if (tid == 0) {
        const double tt = 2.0 * 3.14159265358979323846 * Wsh[4];
        const double pref_d = Wsh[0] / (tt * sqrt(tt));
        double lam[5];
        for (int i = 0; i < 5; ++i) lam[i] = Ush[i] / (pref_d * w3) - Gsh[0][i];
        solve5(Gsh, lam);
        const double nu = a.nu_density ? a.nu * Wsh[0] : a.nu;
        par[0] = pref_d;
        par[1] = nu;
        par[2] = MODE == 2 ? exp(-nu * a.dt) : nu * a.dt;
        for (int i = 0; i < 5; ++i) par[3 + i] = lam[i];
      }
      __syncthreads();
      const R pref = R(par[0]), nu_c = R(par[1]), rate = R(par[2]);
      const R l1 = R(par[4]), l4 = R(par[7]);
      const R Lr = R(a.L), dvr = R(dv);
      const R rz = -Lr + R(iz) * dvr;
      // per y half: the factors that do not depend on v_x
      R pyz[H], cyz[H];
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const int iy = iy0 + h * YH;
        const R ry = -Lr + R(iy) * dvr;
        pyz[h] = pref * gr[N + iy] * gr[2 * N + iz];
        cyz[h] = R(1) + R(par[3]) + R(par[5]) * ry + R(par[6]) * rz + l4 * (R(0.5) * (ry * ry + rz * rz));
      }
      double mom[5] = {0, 0, 0, 0, 0};
#pragma unroll 1
      for (int u0 = 0; u0 < VPT; u0 += B) {
        T xs[B];
#pragma unroll
        for (int j = 0; j < B; ++j) xs[j] = STAGE ? stage[(u0 + j) * NTH + tcell] : load_shifted(u0 + j);
#pragma unroll
        for (int j = 0; j < B; ++j) {
          const int h = j % H, ix = ((u0 + j) / H) * MM + ix0, k = (u0 + j) * NTH + tcell;
          const R rx = -Lr + R(ix) * dvr;
          const R corr = cyz[h] + l1 * rx + l4 * (R(0.5) * (rx * rx));
          const R E = pyz[h] * gr[ix] * corr;
          const R x = xs[j];
          const T out = MODE == 2 ? E + (x - E) * rate : x + rate * (E - x);
          fo[uint32_t(k)] = out;
          if constexpr (EXTRAS) {
            if (q) q[size_t(cell) * NV + k] = nu_c * (E - x);
            if (a.moments) {
              const double d = double(out);
              const double vx = -a.L + double(ix) * dv, vy = -a.L + double(iy0 + h * YH) * dv;
              mom[0] += d;
              mom[1] += d * vx;
              mom[2] += d * vy;
              mom[3] += d * vz;
              mom[4] += d * (0.5 * (vx * vx + vy * vy + vz * vz));
            }
          }
        }
      }
      if (EXTRAS && a.moments) {
        block_sum5(mom, red);
        if (tid == 0)
          for (int i = 0; i < 5; ++i) a.moments[size_t(cell) * 5 + i] = mom[i] * w3;
      }
    }
    __syncthreads();  // the per-cell tables are rewritten for the next cell
  }
}

// Normalised non-equilibrium residual of each cell's f (the macroscopic moments of
// Section 3 one order further): with rho, u, T of f, the deviatoric stress
// sigma_ij = sum f c_i c_j dv^3 - rho T delta_ij and the heat flux q_i = 1/2 sum f |c|^2 c_i dv^3
// (c = v - u) vanish for a Maxwellian; r = |sigma|_F / (rho T) + |q| / (rho T^{3/2}).  One
// workgroup per cell, FP64 sums of the raw moments (1, v, v v, |v|^2 v) in one pass, the
// central ones formed from them.
__global__ __launch_bounds__(256) void k_noneq(const void* __restrict__ fv, int is_f32, int n, double L,
                                               double* __restrict__ r_out) {
  __shared__ double red[13 * 4];
  const int cell = blockIdx.x, nv = n * n * n, tid = threadIdx.x;
  const double dv = 2.0 * L / n;
  double m[13] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};   // 1, v(3), vv(6: xx yy zz xy xz yz), |v|^2 v(3)
  for (int k = tid; k < nv; k += blockDim.x) {
    const double x = is_f32 ? double(static_cast<const float*>(fv)[size_t(cell) * nv + k])
                            : static_cast<const double*>(fv)[size_t(cell) * nv + k];
    const double vx = -L + double(k / (n * n)) * dv, vy = -L + double((k / n) % n) * dv, vz = -L + double(k % n) * dv;
    const double v2 = vx * vx + vy * vy + vz * vz;
    m[0] += x;
    m[1] += x * vx;
    m[2] += x * vy;
    m[3] += x * vz;
    m[4] += x * vx * vx;
    m[5] += x * vy * vy;
    m[6] += x * vz * vz;
    m[7] += x * vx * vy;
    m[8] += x * vx * vz;
    m[9] += x * vy * vz;
    m[10] += x * v2 * vx;
    m[11] += x * v2 * vy;
    m[12] += x * v2 * vz;
  }
  const int lane = tid & 63, wid = tid >> 6;
  for (int i = 0; i < 13; ++i) {
    double v = m[i];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[i * 4 + wid] = v;
  }
  __syncthreads();
  if (tid != 0) return;
  const double w = dv * dv * dv;
  double M[13];
  for (int i = 0; i < 13; ++i) M[i] = w * (red[i * 4] + red[i * 4 + 1] + red[i * 4 + 2] + red[i * 4 + 3]);
  const double rho = M[0];
  const double u[3] = {M[1] / rho, M[2] / rho, M[3] / rho};
  const double M2[3][3] = {{M[4], M[7], M[8]}, {M[7], M[5], M[9]}, {M[8], M[9], M[6]}};
  double P[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) P[i][j] = M2[i][j] - rho * u[i] * u[j];
  const double T = (P[0][0] + P[1][1] + P[2][2]) / (3.0 * rho);
  double s2 = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const double sg = P[i][j] - (i == j ? rho * T : 0.0);
      s2 += sg * sg;
    }
  // sum f |c|^2 c_i = M3_i - u_i tr(M2) - 2 (M2 u)_i + 2 rho |u|^2 u_i
  const double tr = M[4] + M[5] + M[6], uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  double q2 = 0.0;
  for (int i = 0; i < 3; ++i) {
    const double mu = M2[i][0] * u[0] + M2[i][1] * u[1] + M2[i][2] * u[2];
    const double qi = 0.5 * (M[10 + i] - u[i] * tr - 2.0 * mu + 2.0 * rho * uu * u[i]);
    q2 += qi * qi;
  }
  r_out[cell] = sqrt(s2) / (rho * T) + sqrt(q2) / (rho * T * sqrt(T));
}

hipError_t launch_noneq(int dtype_is_f32, int n, const void* f, int64_t cells, double L, double* r, void* stream) {
  if (cells <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_noneq, dim3(unsigned(cells)), dim3(256), 0, static_cast<hipStream_t>(stream), f,
                     dtype_is_f32, n, L, r);
  return hipGetLastError();
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

hipError_t launch_xport_reset(const XportState& st, int n, void* stream) {
  const int m = 3 * n * n * n;
  hipLaunchKernelGGL(k_xport_reset, dim3((m + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream), st.s,
                     st.o, st.dl, st.d1, m, 3 * n);
  return hipGetLastError();
}

hipError_t launch_xport_advance(const XportState& st, int n, double L, double dt, double dx, void* stream) {
  const int nv = n * n * n;
  prof_mark(kProfAdvance, true, static_cast<hipStream_t>(stream));
  hipLaunchKernelGGL(k_xport_advance, dim3((nv + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream),
                     st.s, st.o, st.dl, st.d1, n, L, dt, dx);
  prof_mark(kProfAdvance, false, static_cast<hipStream_t>(stream));
  return hipGetLastError();
}

hipError_t launch_clear_pending(int32_t* d1, int n, void* stream) {
  hipLaunchKernelGGL(k_clear_pending, dim3(1), dim3(3 * n <= 1024 ? 3 * n : 1024), 0,
                     static_cast<hipStream_t>(stream), d1, 3 * n);
  return hipGetLastError();
}

// mode: 0 DM update + shift, 1 DM + Euler BGK, 2 DM + exact BGK, 3 shift only
static hipError_t launch_cell_step(int dtype_is_f32, const void* fin, void* fout, const int32_t* d1, int mode,
                                   const StepCellArgs& a, hipStream_t st) {
  const int64_t cells = int64_t(a.nx) * a.ny * a.nz;
  if (mode != 3 && !a.cons) return hipErrorInvalidValue;
  auto go = [&](auto tag, auto nc) -> hipError_t {
    using T = decltype(tag);
    constexpr int NN = decltype(nc)::value;
    constexpr int NTH = CellShape<T, NN>::NTH;
    // one workgroup per cell, in rounds of at most 2^32 / NTH work-items; a multiple of 8
    // workgroups so that each XCD gets the same share of every round
    const int64_t cap = ((int64_t(1) << 31) / NTH) & ~int64_t(7);
    const int64_t want = (cells + 7) & ~int64_t(7);
    const dim3 grid(unsigned(want < cap ? want : cap)), block(NTH);
    const T* fi = static_cast<const T*>(fin);
    T* fo = static_cast<T*>(fout);
    const bool extras = a.q || a.moments;
    // LDS for the BGK modes' staged masses (see STAGE in the kernel)
    constexpr size_t cb = size_t(CellShape<T, NN>::NV) * sizeof(T);
    constexpr size_t sl = cb <= 64 * 1024 ? cb : 0;
    switch (mode) {
      case 0: hipLaunchKernelGGL((k_cell_step<T, NN, 0, false>), grid, block, 0, st, fi, fo, d1, a); break;
      case 1:
        if (extras) hipLaunchKernelGGL((k_cell_step<T, NN, 1, true>), grid, block, sl, st, fi, fo, d1, a);
        else hipLaunchKernelGGL((k_cell_step<T, NN, 1, false>), grid, block, sl, st, fi, fo, d1, a);
        break;
      case 2:
        if (extras) hipLaunchKernelGGL((k_cell_step<T, NN, 2, true>), grid, block, sl, st, fi, fo, d1, a);
        else hipLaunchKernelGGL((k_cell_step<T, NN, 2, false>), grid, block, sl, st, fi, fo, d1, a);
        break;
      case 3: hipLaunchKernelGGL((k_cell_step<T, NN, 3, false>), grid, block, 0, st, fi, fo, d1, a); break;
      default: return hipErrorInvalidValue;
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
  return dtype_is_f32 ? by_n(float{}) : by_n(double{});
}

hipError_t launch_roll(int dtype_is_f32, const void* fin, void* fout, int32_t* d1, int n, double L, int nx,
                       int ny, int nz, void* stream) {
  StepCellArgs a{};
  a.n = n;
  a.L = L;
  a.nx = nx;
  a.ny = ny;
  a.nz = nz;
  hipStream_t st = static_cast<hipStream_t>(stream);
  prof_mark(kProfRoll, true, st);
  hipError_t e = launch_cell_step(dtype_is_f32, fin, fout, d1, 3, a, st);
  prof_mark(kProfRoll, false, st);
  if (e == hipSuccess) e = launch_clear_pending(d1, n, stream);
  return e;
}

hipError_t launch_step_cell(int dtype_is_f32, const void* fin, void* fout, int32_t* d1, int mode,
                            const StepCellArgs& a, void* stream) {
  if (mode < 0 || mode > 2) return hipErrorInvalidValue;
  hipStream_t st = static_cast<hipStream_t>(stream);
  prof_mark(kProfRoll, true, st);
  hipError_t e = launch_cell_step(dtype_is_f32, fin, fout, d1, mode, a, st);
  prof_mark(kProfRoll, false, st);
  if (e == hipSuccess) e = launch_clear_pending(d1, a.n, stream);
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
