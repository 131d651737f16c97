// Batched fast spectral collision operator Q(f, f) on gfx950 (Appendix A of the paper):
// kernels and their templated launchers, compiled once per precision
// (fks_collide_f32.hip, fks_collide_f64.hip).
//
// Per cell the operator is evaluated as
//   fhat = DFT_n(f) / n^3 on the symmetric mode set K = {-n/2+1 .. n/2-1}^3      (kernel 1)
//   for every separable term t (M directions [x radial nodes] plus the loss):
//     Z_t = IDFT_P[ pad_P( (alpha_t + i alpha'_t) fhat ) ],   G += Re Z_t * Im Z_t (kernel 2)
//   Qhat = DFT_P(G) / P^3 restricted to K;  Q = IDFT_n(Qhat)                       (kernel 3)
// with P = 3n/2 (linear convolution on the kept modes, i.e. the Galerkin-truncated
// sum of eq. CF1).  alpha_t and alpha'_t are real and even and fhat is Hermitian, so
// Re Z_t and Im Z_t are the two real convolution factors of term t.
//
// Kernel 2 splits the padded grid of one cell into S slabs of Z = P/S z-planes,
// slab r owning the planes z = r + S z'.  The first (z) inverse pass of each slab is
// the radix-S decimation-in-frequency step folded into the input: every mode k_z is
// multiplied by exp(2 pi i k_z r / P) and accumulated into bin k_z mod Z, followed by a
// Z-point inverse DFT.  The remaining y and x passes run on the slab's planes only,
// staged through LDS; each thread keeps its part of the slab's G in registers.  At the end the slab
// applies the forward x and y passes (real input, kept modes only) and a Z-point forward
// DFT over its planes; kernel 3 combines the S slab partials with exp(-2 pi i k_z r / P)
// (the matching decimation-in-time step), synthesises Q on the velocity grid and runs
// the FP64 epilogue (conservation projection, Euler update, moments).
#pragma once

#include <hip/hip_runtime.h>

#include "fks_fft.hpp"
#include "fks_internal.hpp"

namespace fks {

// Compiled slab schedules per (precision, n): the number of slabs S per cell (the
// autotuner picks one at run time).  Each of the 2*Z*P threads of a slab owns half an x
// line (P/2 values of one parity) of the slab accumulator G in registers; the LDS holds
// two stage buffers of Z planes, so S is the smallest divisor of P with Z = P/S planes of
// both buffers within the 160 KB of a CU (FP64 needs twice the slabs of FP32).
template <typename T, int N>
struct Variants;
template <int N>
struct Variants<float, N> {
  static constexpr int count = (N >= 16) ? 2 : 1;
  static constexpr int s[2] = {N >= 24 ? 6 : (N >= 16 ? 3 : 1), N >= 32 ? 8 : (N >= 24 ? 9 : 6)};
};
template <int N>
struct Variants<double, N> {
  // n = 16 also has a 6-slab schedule: more workgroups per cell cut the latency of small
  // batches (a single space-homogeneous cell)
  static constexpr int count = (N == 16) ? 2 : 1;
  static constexpr int s[2] = {N >= 32 ? 12 : (N >= 24 ? 6 : (N >= 16 ? 3 : 1)), N == 16 ? 6 : 0};
};

// Grid constants shared by all schedules of (precision, n).
template <typename T, int N>
struct Grid {
  static constexpr int P = 3 * N / 2;
  static constexpr int K = N - 1;
  static constexpr int Kh = N / 2 - 1;
  static constexpr int KH1 = Kh + 1;
  static constexpr int WS = P + 1;
  static constexpr int NPAIR = (K * K + 1) / 2;  // z pencils (kx, ky) of the half plane
  static constexpr int rows_for(int S) { return ((N + (P / S) - 1) / (P / S)) * (P / S); }
  // fhat / table layout rows: k_z = row - N/2; row 0 (the dropped Nyquist mode) and rows
  // >= N are zero; enough rows for the chunking of every compiled schedule
  static constexpr int NRL = rows_for(Variants<T, N>::s[0]) > (Variants<T, N>::count > 1 ? rows_for(Variants<T, N>::s[1]) : 0)
                                 ? rows_for(Variants<T, N>::s[0])
                                 : rows_for(Variants<T, N>::s[1]);
};

template <typename T, int N, int S_>
struct Cfg : Grid<T, N> {
  using G_ = Grid<T, N>;
  static constexpr int P = G_::P, K = G_::K, Kh = G_::Kh, KH1 = G_::KH1, WS = G_::WS, NPAIR = G_::NPAIR;
  static constexpr int NRL = G_::NRL;
  static constexpr int S = S_;
  static constexpr int Z = P / S;
  static constexpr int LINES = Z * P;  // x lines (z', y) of the slab
  static constexpr int NCH = (N + Z - 1) / Z;  // k_z chunks of the fold period Z
  // half chunks of stage-1 loads in flight per thread (FP32: four, i.e. two chunks; FP64:
  // two, its registers hold twice the bytes)
  static constexpr int DEPTH = sizeof(T) == 4 ? 4 : 2;
  // the first loads of stage 1 of term t+1 are in flight while the thread runs its
  // stage-3 x line of term t (FP64 5 % faster than stage 1 after stage 3)
  static constexpr bool OVERLAP = true;
  // the y and x lines of stages 2 and 3 are split into XP interleaved parts of P/XP
  // outputs, one thread each (halves; quarters measured no faster in FP64)
  static constexpr int XP = 2;
  // the forward x and y passes after the last term also run in line parts (FP64: a whole
  // P-point line of doubles does not fit the registers of a 512-thread workgroup; FP32
  // keeps one thread per line)
  static constexpr bool FWD_PARTS = sizeof(T) == 8;
  // plain schedule: one thread per line part and at least one per stage-1 pencil
  static constexpr int NT_ = XP * LINES > NPAIR ? XP * LINES : NPAIR;
  static constexpr int NT_PLAIN = (NT_ + 63) / 64 * 64;
  // Producer/consumer wave split (FP32): the first PW waves own the stage-1 pencils (f̂ kept
  // in registers over all terms, one table load per row) and the stage-2 y lines; CT more
  // threads own IPC stage-3 x-line parts each and their part of G, the x lines being taken
  // in XP3 interleaved parts of P/XP3 outputs.  Used where the parts come in equal whole
  // shares of at most three, each wave's parts lie in one part index (LINES a multiple of
  // 64), and the workgroup stays within 1024 threads.
  static constexpr int PW = ((NPAIR + 63) / 64 > (XP * Z * K + 63) / 64) ? (NPAIR + 63) / 64 : (XP * Z * K + 63) / 64;
  static constexpr int XP3 = 4;
  // the fewest consumer threads (a multiple of 64) that take the parts in shares of three
  static constexpr int CT = (XP3 * LINES + 3 * 64 - 1) / (3 * 64) * 64;
  static constexpr bool SPLIT = sizeof(T) == 4 && 64 * PW + CT <= 1024 && P % XP3 == 0 &&
                                (XP3 * LINES) % CT == 0 && (XP3 * LINES) / CT <= 3 && LINES % 64 == 0;
  static constexpr int IPC = SPLIT ? XP3 * LINES / CT : 0;
  static constexpr int NT = SPLIT ? 64 * PW + CT : NT_PLAIN;
  // table rows in flight per producer thread; folded values per group of consumer LDS reads
  static constexpr int PD = 8;
  static constexpr int PIN = 3;
  static constexpr int VG = 1;
  // split schedule, stage 2: y lines in quarters over all NT threads (4 x 256 slots) instead
  // of halves over the producers
  static constexpr bool S2Q = false;
  // plain schedule, FP64: f̂ rows 1 .. RES of the thread's pencil stay in registers for all
  // terms (chunk-twiddled), so stage 1 loads only their table rows; row 0 (the dropped
  // Nyquist mode) is neither loaded nor accumulated
  static constexpr int RES = (sizeof(T) == 8 && N == 32) ? 16 : 0;
  static constexpr size_t w_elems = size_t(Z) * K * WS;
  static constexpr size_t w_bytes = w_elems * sizeof(cpx<T>);
  // stage 1's output buffer [Z][K][K] beside W (double buffering across terms)
  static constexpr size_t x_bytes = size_t(Z) * K * K * sizeof(cpx<T>);
  // after the last term: G staged as [LINES][P] reals, then its x spectra [Z][KH1][WS]
  // row stride of the staged G lines: P + 2 values keeps the rows 8-byte aligned and
  // spreads the lanes of a wave (one line each) over the LDS banks; with stride P = 48 a
  // wave's 64 lanes fall into 4 banks
  static constexpr int GS = P + 2;
  static constexpr size_t gst_bytes = ((size_t(LINES) * GS * sizeof(T) + 255) / 256) * 256;
  static constexpr size_t spec_bytes = size_t(Z) * KH1 * WS * sizeof(cpx<T>);
  static constexpr size_t lds_bytes =
      (w_bytes + x_bytes > gst_bytes + spec_bytes) ? w_bytes + x_bytes : gst_bytes + spec_bytes;
  static_assert(P % S == 0, "slab count must divide P");
  static_assert(P % 2 == 0, "half lines need an even P");
  static_assert(NCH * Z <= NRL, "layout rows too few for this schedule");
  static_assert(lds_bytes <= 160 * 1024, "slab stage buffer exceeds LDS");
  static_assert(NT <= 1024, "too many threads per slab");
};

// Raw buffer loads: one 32-bit per-lane offset plus a scalar offset per access, so an
// unrolled sequence of strided loads needs no per-load 64-bit address registers.
// Accesses beyond num_records bytes return 0 instead of faulting.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, int(bytes), 0x00020000);
}
template <typename T>
__device__ __forceinline__ cpx<T> bload2(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(cpx<T>, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  } else {
    return __builtin_bit_cast(cpx<T>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
  }
}

__device__ __forceinline__ int opaque_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// Half-plane z pencils: p < Kh*K -> kx = 1 + p/K, ky = p%K - Kh;  else kx = 0, ky = p - Kh*K.
// Together with their mirrors (-kx, -ky) they cover all K^2 pencils once.
template <int K, int Kh>
__device__ __forceinline__ void pair_kxy(int p, int& kx, int& ky) {
  if (p < Kh * K) {
    kx = 1 + p / K;
    ky = p % K - Kh;
  } else {
    kx = 0;
    ky = p - Kh * K;
  }
}

// ------------------------------------------------------------------------------------
// kernel 1: fhat = DFT_n(f)/n^3 on the kept modes, stored for the half-plane pencils
// only (the rest is the complex conjugate), layout [kz][pencil] so that a wavefront of
// pencil threads reads one contiguous row per k_z.
template <typename T, int N>
__global__ __launch_bounds__(256) void k_forward_f(const T* __restrict__ f, cpx<T>* __restrict__ fhat,
                                                   cpx<T>* __restrict__ scratch) {
  using C = Grid<T, N>;
  constexpr int K = C::K, Kh = C::Kh, NPAIR = C::NPAIR;
  const int cell = blockIdx.x;
  const T* fc = f + size_t(cell) * N * N * N;
  cpx<T>* sc = scratch + size_t(cell) * N * N * N;
  cpx<T>* fh = fhat + size_t(cell) * C::NRL * NPAIR;
  // z pass: [x][y][z] real -> sc[x][y][kz]
  for (int it = threadIdx.x; it < N * N; it += blockDim.x) {
    cpx<T> a[N];
    const T* row = fc + size_t(it) * N;
    static_for<0, N>([&](auto z) { a[z] = cpx<T>{row[z], T(0)}; });
    dft<N, -1>(a);
    static_for<0, K>([&](auto kz) { sc[size_t(it) * K + kz] = a[(decltype(kz)::value - Kh + N) % N]; });
  }
  __syncthreads();
  // y pass: columns (x, kz)
  for (int it = threadIdx.x; it < N * K; it += blockDim.x) {
    const int x = it / K, kz = it % K;
    cpx<T> a[N];
    static_for<0, N>([&](auto y) { a[y] = sc[(size_t(x) * N + y) * K + kz]; });
    dft<N, -1>(a);
    static_for<0, K>([&](auto ky) {
      sc[(size_t(x) * N + ky) * K + kz] = a[(decltype(ky)::value - Kh + N) % N];
    });
  }
  __syncthreads();
  // x pass: columns (ky, kz) -> half-plane pencils of fhat
  constexpr T scale = T(1.0 / (double(N) * N * N));
  for (int it = threadIdx.x; it < K * K; it += blockDim.x) {
    const int kyi = it / K, kzi = it % K;
    const int ky = kyi - Kh;
    cpx<T> a[N];
    static_for<0, N>([&](auto x) { a[x] = sc[(size_t(x) * N + kyi) * K + kzi]; });
    dft<N, -1>(a);
    static_for<0, Kh + 1>([&](auto kxv) {
      constexpr int kx = decltype(kxv)::value;
      if (kx > 0 || ky >= 0) {
        const int p = kx > 0 ? (kx - 1) * K + kyi : Kh * K + ky;
        const cpx<T> v = a[kx];
        fh[size_t(kzi + 1) * NPAIR + p] = cpx<T>{v.re * scale, v.im * scale};
      }
    });
  }
  // zero rows: the Nyquist mode k_z = -N/2 and the chunk padding
  for (int i = threadIdx.x; i < NPAIR; i += blockDim.x) fh[i] = cpx<T>{T(0), T(0)};
  for (int i = threadIdx.x; i < (C::NRL - N) * NPAIR; i += blockDim.x) fh[size_t(N) * NPAIR + i] = cpx<T>{T(0), T(0)};
}

// LDS-resident forward transform: the real z rows are reduced to k_z = 0..N/2-1 (the
// negative k_z follow by Hermitian symmetry), so one cell's partial spectra
// [x][y][k_z] (row stride padded by one) fit in LDS and f is read once, fhat written once.
template <typename T, int N>
struct FwdLds {
  static constexpr int KH1 = N / 2;
  static constexpr int RS = KH1 + 1;
  static constexpr size_t bytes = size_t(N) * N * RS * sizeof(cpx<T>);
  static constexpr bool fits = bytes <= 156 * 1024;
};

template <typename T, int N>
__global__ __launch_bounds__(512) void k_forward_lds(const T* __restrict__ f, cpx<T>* __restrict__ fhat) {
  using C = Grid<T, N>;
  using F = FwdLds<T, N>;
  constexpr int K = C::K, Kh = C::Kh, KH1 = F::KH1, RS = F::RS, NPAIR = C::NPAIR, H = N / 2;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  cpx<T>* sm = reinterpret_cast<cpx<T>*>(lds_raw);
  const int cell = blockIdx.x;
  const T* fc = f + size_t(cell) * N * N * N;
  cpx<T>* fh = fhat + size_t(cell) * C::NRL * NPAIR;
  const int tid = threadIdx.x, nt = blockDim.x;
  // z pass: real rows (x, y) -> k_z = 0..N/2-1
  for (int it = tid; it < N * N; it += nt) {
    T r[N];
    const T* row = fc + size_t(it) * N;
    static_for<0, N>([&](auto z) { r[z] = row[z]; });
    cpx<T> o[KH1];
    rdft_low<N, KH1>(r, o);
    static_for<0, KH1>([&](auto kz) { sm[size_t(it) * RS + kz] = o[kz]; });
  }
  __syncthreads();
  // y pass: columns (x, k_z), in place y -> k_y index k_y + Kh
  for (int it = tid; it < N * KH1; it += nt) {
    const int x = it / KH1, kz = it % KH1;
    cpx<T> a[N];
    static_for<0, N>([&](auto y) { a[y] = sm[(size_t(x) * N + y) * RS + kz]; });
    dft<N, -1>(a);
    static_for<0, K>([&](auto kyi) {
      sm[(size_t(x) * N + kyi) * RS + kz] = a[(decltype(kyi)::value - Kh + N) % N];
    });
  }
  __syncthreads();
  // x pass: lines (k_y, k_z >= 0); each value goes to its half-plane pencil, directly or
  // (k_z > 0) as the conjugate of the mirrored mode (-k_x, -k_y, -k_z)
  constexpr T scale = T(1.0 / (double(N) * N * N));
  for (int it = tid; it < KH1 * K; it += nt) {
    const int kz = it / K, kyi = it % K;
    const int ky = kyi - Kh;
    cpx<T> a[N];
    static_for<0, N>([&](auto x) { a[x] = sm[(size_t(x) * N + kyi) * RS + kz]; });
    dft<N, -1>(a);
    static_for<0, K>([&](auto kxi) {
      constexpr int kx = decltype(kxi)::value - Kh;
      const cpx<T> v = a[(kx + N) % N];
      const cpx<T> sv = {v.re * scale, v.im * scale};
      const bool direct = kx > 0 || (kx == 0 && ky >= 0);
      if (direct) {
        const int p = kx > 0 ? (kx - 1) * K + kyi : Kh * K + ky;
        fh[size_t(kz + H) * NPAIR + p] = sv;
        if (kx == 0 && ky == 0 && kz > 0) fh[size_t(H - kz) * NPAIR + p] = conj(sv);
      } else if (kz > 0) {
        const int mkx = -kx, mky = -ky;  // (mkx, mky) lies in the half plane
        const int p = mkx > 0 ? (mkx - 1) * K + (mky + Kh) : Kh * K + mky;
        fh[size_t(H - kz) * NPAIR + p] = conj(sv);
      }
    });
  }
  // zero rows: the Nyquist mode k_z = -N/2 and the chunk padding
  for (int i = tid; i < NPAIR; i += nt) fh[i] = cpx<T>{T(0), T(0)};
  for (int i = tid; i < (C::NRL - N) * NPAIR; i += nt) fh[size_t(N) * NPAIR + i] = cpx<T>{T(0), T(0)};
}

// Forward transform in two k_z passes for cells whose partial spectra exceed the LDS (FP64
// n = 32): pass p reduces the real z rows to the modes k_z = p KB .. p KB + KB - 1 of
// 0..N/2-1, runs the y and x passes on them in LDS and writes their pencils; f is read once
// per pass (the second time mostly from the caches), fhat written once.
template <typename T, int N>
struct FwdSplit {
  static constexpr int KH1 = N / 2;
  static constexpr int KB = KH1 / 2;
  static constexpr int RS = KB + 1;
  static constexpr size_t bytes = size_t(N) * N * RS * sizeof(cpx<T>);
  static constexpr bool fits = bytes <= 156 * 1024;
};

template <typename T, int N>
__global__ __launch_bounds__(512) void k_forward_split(const T* __restrict__ f, cpx<T>* __restrict__ fhat) {
  using C = Grid<T, N>;
  using F = FwdSplit<T, N>;
  constexpr int K = C::K, Kh = C::Kh, KH1 = F::KH1, KB = F::KB, RS = F::RS, NPAIR = C::NPAIR, H = N / 2;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  cpx<T>* sm = reinterpret_cast<cpx<T>*>(lds_raw);
  const int cell = blockIdx.x;
  const T* fc = f + size_t(cell) * N * N * N;
  cpx<T>* fh = fhat + size_t(cell) * C::NRL * NPAIR;
  const int tid = threadIdx.x, nt = blockDim.x;
  constexpr T scale = T(1.0 / (double(N) * N * N));
  static_for<0, 2>([&](auto pc) {
    constexpr int kz0 = decltype(pc)::value * KB;
    // z pass: real rows (x, y) -> the pass's KB modes
    for (int it = tid; it < N * N; it += nt) {
      T r[N];
      const T* row = fc + size_t(it) * N;
      static_for<0, N>([&](auto z) { r[z] = row[z]; });
      cpx<T> o[KH1];
      rdft_low<N, KH1>(r, o);
      static_for<0, KB>([&](auto j) { sm[size_t(it) * RS + j] = o[kz0 + decltype(j)::value]; });
    }
    __syncthreads();
    // y pass: columns (x, j), in place y -> k_y index k_y + Kh
    for (int it = tid; it < N * KB; it += nt) {
      const int x = it / KB, j = it % KB;
      cpx<T> a[N];
      static_for<0, N>([&](auto y) { a[y] = sm[(size_t(x) * N + y) * RS + j]; });
      dft<N, -1>(a);
      static_for<0, K>([&](auto kyi) {
        sm[(size_t(x) * N + kyi) * RS + j] = a[(decltype(kyi)::value - Kh + N) % N];
      });
    }
    __syncthreads();
    // x pass: lines (k_y, k_z) as in the LDS-resident kernel
    for (int it = tid; it < KB * K; it += nt) {
      const int j = it / K, kyi = it % K;
      const int kz = kz0 + j, ky = kyi - Kh;
      cpx<T> a[N];
      static_for<0, N>([&](auto x) { a[x] = sm[(size_t(x) * N + kyi) * RS + j]; });
      dft<N, -1>(a);
      static_for<0, K>([&](auto kxi) {
        constexpr int kx = decltype(kxi)::value - Kh;
        const cpx<T> v = a[(kx + N) % N];
        const cpx<T> sv = {v.re * scale, v.im * scale};
        const bool direct = kx > 0 || (kx == 0 && ky >= 0);
        if (direct) {
          const int p = kx > 0 ? (kx - 1) * K + kyi : Kh * K + ky;
          fh[size_t(kz + H) * NPAIR + p] = sv;
          if (kx == 0 && ky == 0 && kz > 0) fh[size_t(H - kz) * NPAIR + p] = conj(sv);
        } else if (kz > 0) {
          const int mkx = -kx, mky = -ky;
          const int p = mkx > 0 ? (mkx - 1) * K + (mky + Kh) : Kh * K + mky;
          fh[size_t(H - kz) * NPAIR + p] = conj(sv);
        }
      });
    }
    __syncthreads();  // the next pass overwrites the LDS
  });
  for (int i = tid; i < NPAIR; i += nt) fh[i] = cpx<T>{T(0), T(0)};
  for (int i = tid; i < (C::NRL - N) * NPAIR; i += nt) fh[size_t(N) * NPAIR + i] = cpx<T>{T(0), T(0)};
}


// ------------------------------------------------------------------------------------
// kernel 2: one slab of one cell, all separable terms

// After the last term of a slab: G, staged in LDS as [LINES][GS] reals at the start of the
// buffer, goes through the forward x pass (real lines (z', y) -> k_x in [0, Kh] ->
// W[z'][kx][y]; part h of a line takes the modes kx = XP j + h), the forward y pass and the
// Z-point DFT over the slab planes, whose result is the slab's partial spectrum D[kx][ky][b]
template <typename T, int N, int S>
__device__ __forceinline__ void slab_forward(cpx<T>* W, cpx<T>* __restrict__ D) {
  using C = Cfg<T, N, S>;
  constexpr int P = C::P, K = C::K, Kh = C::Kh, KH1 = C::KH1, WS = C::WS, Z = C::Z;
  constexpr int NT = C::NT, XP = C::XP, PX = P / XP;
  const int tid = threadIdx.x;
  T* Gst = reinterpret_cast<T*>(W);
  cpx<T>* Wspec = reinterpret_cast<cpx<T>*>(reinterpret_cast<unsigned char*>(W) + C::gst_bytes);
  __syncthreads();
  if constexpr (!C::FWD_PARTS) {
    // FP32: one thread per whole line (packed real transform)
    for (int it = tid; it < C::LINES; it += NT) {
      const int zp = it / P, y = it % P;
      cpx<T> o[KH1];
      rdft_low<P, KH1>(Gst + size_t(it) * C::GS, o);
      static_for<0, KH1>([&](auto kx) { Wspec[(size_t(zp) * KH1 + kx) * WS + y] = o[kx]; });
    }
  } else if (tid < XP * C::LINES) {
    const int h = tid / C::LINES, line = tid - h * C::LINES;
    const int zp = line / P, y = line % P;
    const T* gl = Gst + size_t(line) * C::GS;
    cpx<T> u[PX];
    part_dispatch<XP>(h, [&](auto hc) {
      fold_part_fwd<P, XP, decltype(hc)::value>(u, [&](int i) { return cpx<T>{gl[i], T(0)}; });
    });
    dft<PX, -1>(u);
    static_for<0, PX>([&](auto j) {
      const int kx = XP * decltype(j)::value + h;
      if (kx <= Kh) Wspec[(size_t(zp) * KH1 + kx) * WS + y] = u[j];
    });
  }
  __syncthreads();
  // forward y pass: lines (z', kx) -> ky in K, in place
  if constexpr (!C::FWD_PARTS) {
    for (int it = tid; it < Z * KH1; it += NT) {
      cpx<T>* row = Wspec + size_t(it) * WS;
      cpx<T> a[P];
      static_for<0, P>([&](auto y) { a[y] = row[y]; });
      dft<P, -1>(a);
      static_for<0, K>([&](auto kyi) { row[kyi] = a[(decltype(kyi)::value - Kh + P) % P]; });
    }
  } else {
    // in parts: every part reads its whole line before any part writes its modes back
    constexpr int YL = Z * KH1;
    static_assert(XP * YL <= NT, "one round of line parts");
    const bool act = tid < XP * YL;
    const int h = act ? tid / YL : 0, line = act ? tid - h * YL : 0;
    cpx<T>* row = Wspec + size_t(line) * WS;
    cpx<T> u[PX];
    if (act) part_dispatch<XP>(h, [&](auto hc) { fold_part_fwd<P, XP, decltype(hc)::value>(u, [&](int i) { return row[i]; }); });
    __syncthreads();
    if (act) {
      dft<PX, -1>(u);
      static_for<0, PX>([&](auto j) {
        const int k = XP * decltype(j)::value + h;   // DFT index of the output, signed mode k or k - P
        if (k <= Kh) row[k + Kh] = u[j];
        else if (k >= P - Kh) row[k - P + Kh] = u[j];
      });
    }
  }
  __syncthreads();
  // Z-point forward DFT over the slab planes -> D[kx][ky][b]
  for (int it = tid; it < KH1 * K; it += NT) {
    const int kx = it / K, ky = it % K;
    cpx<T> a[Z];
    static_for<0, Z>([&](auto zp) { a[zp] = Wspec[(size_t(zp) * KH1 + kx) * WS + ky]; });
    dft<Z, -1>(a);
    static_for<0, Z>([&](auto b) { D[size_t(it) * Z + b] = a[b]; });
  }
}

template <typename T, int N, int S, int RID>
__device__ __forceinline__ void slab_body(const cpx<T>* __restrict__ fh, const T* __restrict__ tab,
                                          int n_terms, int t_begin, int t_end, cpx<T>* __restrict__ D,
                                          cpx<T>* W) {
  using C = Cfg<T, N, S>;
  constexpr int P = C::P, K = C::K, Kh = C::Kh, WS = C::WS, Z = C::Z, NPAIR = C::NPAIR;
  constexpr int NT = C::NT;
  const int tid = threadIdx.x;

  // thread tid < XP*LINES owns the line part (h, line) = divmod(tid, LINES) of G, i.e.
  // g[j] = G[line][XP j + h]; h is uniform over all but at most one wavefront
  constexpr int XP = C::XP, PX = P / XP;
  T g[PX];
  static_for<0, PX>([&](auto j) { g[j] = T(0); });
  // u = the XP-part fold of a pruned line (inverse transforms) for the run-time part h
  auto fold = [&](cpx<T>* u, int h, auto&& load) {
    part_dispatch<XP>(h, [&](auto hc) { fold_part<P, XP, Kh, decltype(hc)::value>(u, load); });
  };

  constexpr uint32_t row_bytes = uint32_t(NPAIR) * sizeof(cpx<T>);  // one k_z row, fhat and tables
  const __amdgpu_buffer_rsrc_t rf = make_rsrc(fh, uint32_t(C::NRL) * row_bytes);
  const __amdgpu_buffer_rsrc_t rt = make_rsrc(tab, uint32_t(n_terms) * C::NRL * row_bytes);
  // stage 1 of term t: half-plane pencil p and its mirror.  Mode k_z of pencil (kx, ky)
  // and mode -k_z of (-kx, -ky) come from the same stored value (Hermitian fhat, even
  // tables).  Rows are taken in chunks j of Z consecutive modes; with k_z = jZ + b - N/2
  // the slab twiddle exp(2 pi i k_z r/P) = w_S^{jr} exp(2 pi i (b - N/2) r/P): the chunk
  // factor w_S^{jr} is a compile-time constant (for most (j, r) it is +-1, always at
  // j = 0 and r = 0, and its complex product folds away), the per-bin factor is applied
  // once after the last chunk.  Output: the Z planes [z'][kx + Kh][ky + Kh] of dst with
  // row stride `ld`.
  //
  // The rows are streamed through a software pipeline of DEPTH half chunks: the loads of
  // the next half chunks are in flight while the current one is accumulated.  The
  // pipeline is primed (stage1_issue: the first DEPTH half chunks) before `mid` runs and
  // drained after it (stage1_finish), so that independent work placed in `mid` hides the
  // latency of the first loads.
  constexpr int ZH = (Z + 1) / 2;
  // DEPTH half-chunk slots in flight (a ring over the 2*NCH half chunks)
  constexpr int DEPTH = C::DEPTH < 2 * C::NCH ? C::DEPTH : 2 * C::NCH;
  struct Pipe {
    cpx<T> pf[DEPTH][ZH], pa[DEPTH][ZH];
  };
  // f̂ rows 1 .. RES in registers (C::RES > 0), each times its chunk twiddle w_S^{jr}
  constexpr int RES = C::RES;
  cpx<T> gres[RES > 0 ? RES : 1];
  if constexpr (RES > 0) {
    const uint32_t voff = uint32_t(opaque_tid()) * sizeof(cpx<T>);
    static_for<0, RES>([&](auto i) {
      constexpr int r = decltype(i)::value + 1;
      gres[i] = twiddle<C::S, +1, long(r / Z) * RID>(bload2<T>(rf, voff, uint32_t(r) * row_bytes));
    });
  }
  // rows 0 .. row_live_from - 1 take no f̂ load (zero, or held in gres)
  auto load_half = [&](Pipe& q, uint32_t voff, uint32_t tterm, auto hc) {
    constexpr int h = decltype(hc)::value, slot = h % DEPTH, b0 = (h % 2) * ZH;
    constexpr uint32_t s0 = uint32_t(h / 2) * Z * row_bytes;
    static_for<0, ZH>([&](auto i) {
      constexpr int bb = b0 + decltype(i)::value;
      constexpr int row = (h / 2) * Z + bb;
      if constexpr (bb < Z && !(RES > 0 && row == 0)) {
        if constexpr (!(RES > 0 && row <= RES)) q.pf[slot][i] = bload2<T>(rf, voff, s0 + uint32_t(bb) * row_bytes);
        q.pa[slot][i] = bload2<T>(rt, voff, tterm + s0 + uint32_t(bb) * row_bytes);
      }
    });
  };
  auto stage1_issue = [&](Pipe& q, int p, int t) {
    const uint32_t voff = uint32_t(p) * sizeof(cpx<T>);
    const uint32_t tterm = uint32_t(t) * C::NRL * row_bytes;
    static_for<0, DEPTH>([&](auto hc) { load_half(q, voff, tterm, hc); });
  };
  auto stage1_finish = [&](Pipe& q, int p, int t, cpx<T>* dst, auto ld_c) {
    constexpr int LD = decltype(ld_c)::value;
    const uint32_t voff = uint32_t(p) * sizeof(cpx<T>);
    const uint32_t tterm = uint32_t(t) * C::NRL * row_bytes;
    int kx, ky;
    pair_kxy<K, Kh>(p, kx, ky);
    // With g = w f (w the chunk twiddle) and the real table pair (a, b), the pencil
    // accumulates (a + ib) g and its mirror conj((a - ib) g); both come from the four
    // real sums s1 = sum a Re g, s2 = sum b Im g, s3 = sum a Im g, s4 = sum b Re g:
    // A = (s1 - s2, s3 + s4), B = (s1 + s2, s4 - s3).
    T s1[Z], s2[Z], s3[Z], s4[Z];
    static_for<0, Z>([&](auto bb) {
      s1[bb] = T(0);
      s2[bb] = T(0);
      s3[bb] = T(0);
      s4[bb] = T(0);
    });
    auto accumulate = [&](auto hc) {
      constexpr int h = decltype(hc)::value, slot = h % DEPTH, b0 = (h % 2) * ZH;
      constexpr long qe = long(h / 2) * RID;
      static_for<0, ZH>([&](auto i) {
        constexpr int bb = b0 + decltype(i)::value;
        constexpr int row = (h / 2) * Z + bb;
        if constexpr (bb < Z && !(RES > 0 && row == 0)) {
          const cpx<T> ab = q.pa[slot][i];
          cpx<T> g;
          if constexpr (RES > 0 && row <= RES) g = gres[row - 1];
          else g = twiddle<C::S, +1, qe>(q.pf[slot][i]);
          if constexpr (sizeof(T) == 8) {
            // FP64: sums in program order.  Reassociated, the unrolled chunk products
            // are regrouped by twiddle constant and all kept live (hundreds of spilled
            // registers at S = 12); FP32 keeps the faster reassociated form
#pragma clang fp reassociate(off)
            s1[bb] += ab.re * g.re;
            s2[bb] += ab.im * g.im;
            s3[bb] += ab.re * g.im;
            s4[bb] += ab.im * g.re;
          } else {
            s1[bb] += ab.re * g.re;
            s2[bb] += ab.im * g.im;
            s3[bb] += ab.re * g.im;
            s4[bb] += ab.im * g.re;
          }
        }
      });
    };
    static_for<0, 2 * C::NCH>([&](auto hc) {
      constexpr int h = decltype(hc)::value;
      // no load is hoisted past the half chunk that frees its slot
      sched_fence();
      accumulate(hc);
      if constexpr (h + DEPTH < 2 * C::NCH) load_half(q, voff, tterm, std::integral_constant<int, h + DEPTH>{});
    });
    // per-bin twiddles and the bin of each partial sum (k_z mod Z, resp. -k_z mod Z)
    cpx<T> oA[Z], oB[Z];
    static_for<0, Z>([&](auto bb) {
      constexpr int e = decltype(bb)::value - N / 2;
      const cpx<T> bA = {s1[bb] - s2[bb], s3[bb] + s4[bb]};
      const cpx<T> bB = {s1[bb] + s2[bb], s4[bb] - s3[bb]};
      oA[((e % Z) + Z) % Z] = twiddle<P, +1, long(e) * RID>(bA);
      oB[(((-e) % Z) + Z) % Z] = twiddle<P, +1, -long(e) * RID>(bB);
    });
    dft<Z, +1>(oA);
    const int kxa = kx + Kh, kya = ky + Kh;
    static_for<0, Z>([&](auto zp) { dst[(size_t(zp) * K + kxa) * LD + kya] = oA[zp]; });
    if (kx != 0 || ky != 0) {
      dft<Z, +1>(oB);
      const int kxb = Kh - kx, kyb = Kh - ky;
      static_for<0, Z>([&](auto zp) { dst[(size_t(zp) * K + kxb) * LD + kyb] = oB[zp]; });
    }
  };
  // Every stage takes an opaque copy of the thread index (opaque_tid): its index
  // arithmetic is redone where it is used instead of being hoisted out of the term loop
  // or shared between stages and kept live next to the accumulator (LDS plane offsets
  // beyond the 64 KiB immediate range need their own address registers).
  auto stage1 = [&](int t, cpx<T>* dst, auto ld_c, auto&& mid) {
    // one pencil per thread at most
    static_assert(NPAIR <= NT, "every pencil has its own thread");
    const int p = opaque_tid();
    Pipe q;
    if (p < NPAIR) stage1_issue(q, p, t);
    sched_fence();
    mid();
    sched_fence();
    if (p < NPAIR) stage1_finish(q, p, t, dst, ld_c);
  };
  auto nothing = [] {};

  {
    // two LDS buffers.  X holds stage 1's output [Z][K][K]; W the y-transformed
    // planes [Z][K][P+1].  Per term t: stage 2 reads X(t) and writes W; then, in one
    // barrier interval, stage 1 of term t+1 refills X while stage 3 of term t consumes W,
    // so the waves waiting on stage 1's loads overlap with the others' x-line transforms.
    cpx<T>* X = W + C::w_elems;
    using LdX = std::integral_constant<int, K>;
    if (t_begin < t_end) stage1(t_begin, X, LdX{}, nothing);
    __syncthreads();
    for (int t = t_begin; t < t_end; ++t) {
      // stage 2: y lines (z', kx): K modes -> P points; work item it = h*Z*K + line
      // computes the outputs y = XP j + h of one line
      {
        const int tid = opaque_tid();
        constexpr int HL = Z * K, ITEMS = XP * HL;
        static_assert(ITEMS <= NT, "one round of line parts");
        if (tid < ITEMS) {
          const int h = tid / HL, line = tid - h * HL;
          const cpx<T>* src = X + size_t(line) * K;
          cpx<T>* row = W + size_t(line) * WS;
          cpx<T> u[PX];
          fold(u, h, [&](int i) { return src[i]; });
          dft<PX, +1>(u);
          static_for<0, PX>([&](auto j) { row[XP * decltype(j)::value + h] = u[j]; });
        }
      }
      __syncthreads();
      // stage 3: x lines (z', y): K modes -> P points, G += Re * Im; it runs between the
      // first loads and the accumulation of stage 1 of term t + 1
      auto stage3 = [&] {
        const int tid = opaque_tid();
        if (tid < XP * C::LINES) {
          const int h = tid / C::LINES, line = tid - h * C::LINES;
          const int zp = line / P, y = line % P;
          const cpx<T>* col = W + size_t(zp) * K * WS + y;
          cpx<T> u[PX];
          fold(u, h, [&](int i) { return col[size_t(i) * WS]; });
          dft<PX, +1>(u);
          static_for<0, PX>([&](auto j) { g[j] += u[j].re * u[j].im; });
        }
      };
      if constexpr (C::OVERLAP) {
        if (t + 1 < t_end) stage1(t + 1, X, LdX{}, stage3);
        else stage3();
      } else {
        stage3();
        if (t + 1 < t_end) stage1(t + 1, X, LdX{}, nothing);
      }
      __syncthreads();
    }
  }

  T* Gst = reinterpret_cast<T*>(W);
  if (tid < XP * C::LINES) {
    const int h = tid / C::LINES, line = tid - h * C::LINES;
    static_for<0, PX>([&](auto j) { Gst[size_t(line) * C::GS + XP * decltype(j)::value + h] = g[j]; });
  }
  slab_forward<T, N, S>(W, D);
}

// The same slab computation with the waves split into producers and consumers (C::SPLIT).
// Producer waves keep their pencil's f̂ rows, already multiplied by the slab's chunk
// twiddles, in registers for all terms, so a term's stage 1 reads only its table rows
// (half of the L2 traffic of the plain schedule); they also run stage 2.  Consumer waves
// run stage 3 for IPC x-line parts each and hold those parts of G.  Both sides pass the
// same barriers: stage 1 of term t+1 (producers) and stage 3 of term t (consumers) share
// one barrier interval, as in the plain schedule.
template <typename T, int N, int S, int RID>
__device__ __forceinline__ void slab_body_split(const cpx<T>* __restrict__ fh, const T* __restrict__ tab,
                                                int n_terms, int t_begin, int t_end, cpx<T>* __restrict__ D,
                                                cpx<T>* W) {
  using C = Cfg<T, N, S>;
  constexpr int P = C::P, K = C::K, Kh = C::Kh, WS = C::WS, Z = C::Z, NPAIR = C::NPAIR;
  constexpr int XP = C::XP, PX = P / XP, PW = C::PW, CT = C::CT, IPC = C::IPC, LINES = C::LINES, XP3 = C::XP3;
  static_assert(C::SPLIT, "split schedule only");
  static_assert(XP * Z * K <= 64 * PW && NPAIR <= 64 * PW, "producers cover stage 1 and stage 2");
  static_assert(IPC * CT == XP3 * LINES && CT % 64 == 0, "consumers cover stage 3");
  cpx<T>* X = W + C::w_elems;
  auto fold = [&](cpx<T>* u, int h, auto&& load) {
    part_dispatch<XP>(h, [&](auto hc) { fold_part<P, XP, Kh, decltype(hc)::value>(u, load); });
  };
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  // stage 2 in quarters: slot tid = 256 h + line, part h (outputs y = 4 j + h) of y line
  // `line` < Z K; h is uniform over a wave
  auto stage2q = [&] {
    constexpr int HL = Z * K;
    static_assert(!C::S2Q || (HL <= 256 && C::NT == 1024 && P % 4 == 0), "quarter slots");
    const int tid = opaque_tid();
    const int h = __builtin_amdgcn_readfirstlane(tid >> 8), line = tid & 255;
    if (line < HL) {
      const cpx<T>* src = X + size_t(line) * K;
      cpx<T>* row = W + size_t(line) * WS;
      auto load = [&](int i) {
        int z0 = 0;
        asm volatile("" : "+v"(z0));
        return src[i + z0];
      };
      auto pin = [](const cpx<T>& v, auto kk) {
        if constexpr (decltype(kk)::value % C::PIN == C::PIN - 1) asm volatile("" ::"v"(v.re), "v"(v.im));
      };
      cpx<T> u[P / 4];
      part_dispatch<4>(h, [&](auto hc) { fold_part<P, 4, Kh, decltype(hc)::value>(u, load, pin); });
      dft<P / 4, +1>(u);
      static_for<0, P / 4>([&](auto j) { row[4 * decltype(j)::value + h] = u[j]; });
    }
  };
  if (wave < PW) {
    // ---- producers.  Rows r = 1 .. N-1 of the [row][pencil] layout (k_z = r - N/2; row 0,
    // the dropped Nyquist mode, is zero); row r lies in chunk r / Z, bin r % Z.
    constexpr uint32_t row_bytes = uint32_t(NPAIR) * sizeof(cpx<T>);
    constexpr int NR = N - 1;
    const __amdgpu_buffer_rsrc_t rf = make_rsrc(fh, uint32_t(C::NRL) * row_bytes);
    const __amdgpu_buffer_rsrc_t rt = make_rsrc(tab, uint32_t(n_terms) * C::NRL * row_bytes);
    const int p = opaque_tid();
    const bool act = p < NPAIR;
    // lanes past the last pencil read (and never use) the first pencils of the next row;
    // reads past the end of a buffer return zero
    const uint32_t voff = uint32_t(p) * sizeof(cpx<T>);
    // row r carries the whole slab twiddle exp(2 pi i k_z r_slab / P), k_z = r - N/2: the
    // chunk factor and the per-bin factor of the plain schedule in one (the bin sums then
    // need no twiddle)
    cpx<T> gf[NR];
    static_for<0, NR>([&](auto i) {
      constexpr int r = decltype(i)::value + 1;
      gf[i] = twiddle<P, +1, long(r - N / 2) * RID>(bload2<T>(rf, voff, uint32_t(r) * row_bytes));
    });
    constexpr int PD = C::PD < NR ? C::PD : NR;
    auto stage1 = [&](int t) {
      const uint32_t tterm = uint32_t(t) * C::NRL * row_bytes;
      cpx<T> ta[PD];
      static_for<0, PD>([&](auto i) { ta[i] = bload2<T>(rt, voff, tterm + uint32_t(decltype(i)::value + 1) * row_bytes); });
      uint32_t vo = voff;
      // (a + ib) g and its mirror conj((a - ib) g) from s1 = sum a Re g, s2 = sum b Im g,
      // s3 = sum a Im g, s4 = sum b Re g per bin
      T s1[Z], s2[Z], s3[Z], s4[Z];
      static_for<0, Z>([&](auto bb) {
        s1[bb] = T(0);
        s2[bb] = T(0);
        s3[bb] = T(0);
        s4[bb] = T(0);
      });
      static_for<0, NR>([&](auto i) {
        constexpr int ii = decltype(i)::value, r = ii + 1, bb = r % Z, slot = ii % PD;
        sched_fence();
        const cpx<T> ab = ta[slot];
        const cpx<T> g = gf[ii];
        s1[bb] += ab.re * g.re;
        s2[bb] += ab.im * g.im;
        s3[bb] += ab.re * g.im;
        s4[bb] += ab.im * g.re;
        // the sums of this row are formed before the next load is issued; the loads take an
        // opaque copy of the offset, renewed every C::VG rows, which keeps them in their
        // place in the ring (the loads of read-only memory are otherwise all hoisted to the top)
        if constexpr (ii % C::VG == 0) {
          asm volatile("" : "+v"(vo) : "v"(s1[bb]), "v"(s2[bb]), "v"(s3[bb]), "v"(s4[bb]));
        } else {
          asm volatile("" ::"v"(s1[bb]), "v"(s2[bb]), "v"(s3[bb]), "v"(s4[bb]));
        }
        if constexpr (ii + PD < NR) ta[slot] = bload2<T>(rt, vo, tterm + uint32_t(r + PD) * row_bytes);
      });
      int kx, ky;
      pair_kxy<K, Kh>(act ? p : 0, kx, ky);
      cpx<T> oA[Z], oB[Z];
      static_for<0, Z>([&](auto bb) {
        constexpr int e = decltype(bb)::value - N / 2;
        oA[((e % Z) + Z) % Z] = cpx<T>{s1[bb] - s2[bb], s3[bb] + s4[bb]};
        oB[(((-e) % Z) + Z) % Z] = cpx<T>{s1[bb] + s2[bb], s4[bb] - s3[bb]};
      });
      if (act) {
        dft<Z, +1>(oA);
        const int kxa = kx + Kh, kya = ky + Kh;
        static_for<0, Z>([&](auto zp) { X[(size_t(zp) * K + kxa) * K + kya] = oA[zp]; });
        if (kx != 0 || ky != 0) {
          dft<Z, +1>(oB);
          const int kxb = Kh - kx, kyb = Kh - ky;
          static_for<0, Z>([&](auto zp) { X[(size_t(zp) * K + kxb) * K + kyb] = oB[zp]; });
        }
      }
    };
    if (t_begin < t_end) stage1(t_begin);
    __syncthreads();
    for (int t = t_begin; t < t_end; ++t) {
      if constexpr (C::S2Q) {
        stage2q();
      } else {
        // stage 2: y lines (z', kx) of X -> W, part h of line `line`
        const int tid = opaque_tid();
        constexpr int HL = Z * K;
        if (tid < XP * HL) {
          const int h = tid / HL, line = tid - h * HL;
          const cpx<T>* src = X + size_t(line) * K;
          cpx<T>* row = W + size_t(line) * WS;
          cpx<T> u[PX];
          fold(u, h, [&](int i) { return src[i]; });
          dft<PX, +1>(u);
          static_for<0, PX>([&](auto j) { row[XP * decltype(j)::value + h] = u[j]; });
        }
      }
      __syncthreads();
      if (t + 1 < t_end) stage1(t + 1);
      __syncthreads();
    }
  } else {
    // ---- consumers: x-line part it = c + m CT (m < IPC) of stage 3, i.e. part h = it / LINES
    // (outputs y = XP3 j + h) of line it % LINES; G part g[m]
    constexpr int PX3 = P / XP3;
    T g[IPC][PX3];
    static_for<0, IPC>([&](auto m) { static_for<0, PX3>([&](auto j) { g[m][j] = T(0); }); });
    __syncthreads();
    for (int t = t_begin; t < t_end; ++t) {
      if constexpr (C::S2Q) stage2q();
      __syncthreads();
      const int c = opaque_tid() - 64 * PW;
      static_for<0, IPC>([&](auto m) {
        sched_fence();
        constexpr int mm = decltype(m)::value;
        const int it = c + mm * CT;
        // the CT parts of round mm span the part indices hlo .. hhi (at most two); h is
        // uniform over a wave
        constexpr int hlo = mm * CT / LINES, hhi = (mm * CT + CT - 1) / LINES;
        static_assert(hhi - hlo <= 1, "a round spans at most two part indices");
        const int h = hlo == hhi ? hlo : __builtin_amdgcn_readfirstlane(it / LINES);
        const int line = it - h * LINES;
        const int zp = line / P, y = line % P;
        const cpx<T>* col = W + size_t(zp) * K * WS + y;
        // the LDS reads take an opaque zero offset that is renewed after every C::PIN-th folded
        // value, once that value is formed: the reads of a part are not all hoisted to its top
        // (its 31 inputs, the part and G together exceed the registers)
        int z0 = 0;
        asm volatile("" : "+v"(z0));
        auto load = [&](int i) { return col[size_t(i) * WS + z0]; };
        auto pin = [&z0](const cpx<T>& v, auto kk) {
          if constexpr (decltype(kk)::value % C::PIN == C::PIN - 1) asm volatile("" : "+v"(z0) : "v"(v.re), "v"(v.im));
        };
        cpx<T> u[PX3];
        if (hlo == hhi || h == hlo) fold_part<P, XP3, Kh, hlo>(u, load, pin);
        else fold_part<P, XP3, Kh, hhi>(u, load, pin);
        dft<PX3, +1>(u);
        static_for<0, PX3>([&](auto j) { g[m][j] += u[j].re * u[j].im; });
      });
      __syncthreads();
    }
    // stage G for the forward passes (after the last barrier no part reads W)
    T* Gst = reinterpret_cast<T*>(W);
    const int c = int(threadIdx.x) - 64 * PW;
    static_for<0, IPC>([&](auto m) {
      const int it = c + decltype(m)::value * CT;
      const int h = it / LINES, line = it - h * LINES;
      static_for<0, PX3>([&](auto j) { Gst[size_t(line) * C::GS + XP3 * decltype(j)::value + h] = g[m][j]; });
    });
  }
  slab_forward<T, N, S>(W, D);
}

template <typename T, int N, int S>
__global__ __launch_bounds__((Cfg<T, N, S>::NT)) void k_slab(const cpx<T>* __restrict__ fhat,
                                                           const T* __restrict__ tab, int n_terms,
                                                           cpx<T>* __restrict__ D, int xcd_map, int tg) {
  using C = Cfg<T, N, S>;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  cpx<T>* W = reinterpret_cast<cpx<T>*>(lds_raw);
  // Work unit = (cell, term group g < tg); each unit has S slab workgroups and its own
  // partial D (the finish kernel sums the groups).  Workgroups are dealt round-robin to
  // the 8 XCDs; with xcd_map (tg = 1) the S slabs of one cell land on the same XCD
  // (consecutive in its queue) so they share fhat through its L2.
  const int b = blockIdx.x;
  int unit, r;
  if (xcd_map) {
    const int j = b >> 3;
    unit = (j / C::S) * 8 + (b & 7);
    r = j % C::S;
  } else {
    unit = b / C::S;
    r = b % C::S;
  }
  const int cell = unit / tg, g = unit - cell * tg;
  const int tpg = (n_terms + tg - 1) / tg;
  const int t0 = g * tpg, t1 = t0 + tpg < n_terms ? t0 + tpg : n_terms;
  const cpx<T>* fh = fhat + size_t(cell) * C::NRL * C::NPAIR;
  cpx<T>* Ds = D + (size_t(unit) * C::S + r) * (size_t(C::KH1) * C::K * C::Z);
  static_for<0, C::S>([&](auto rid) {
    if (r == decltype(rid)::value) {
      if constexpr (C::SPLIT) slab_body_split<T, N, S, decltype(rid)::value>(fh, tab, n_terms, t0, t1, Ds, W);
      else slab_body<T, N, S, decltype(rid)::value>(fh, tab, n_terms, t0, t1, Ds, W);
    }
  });
}

// ------------------------------------------------------------------------------------
// kernel 3: combine slabs, synthesise Q on the velocity grid, FP64 epilogue
__device__ __forceinline__ void block_reduce5(double (&v)[5], double* red) {
  // red: LDS [5][NT/64]; result broadcast to all threads
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  static_for<0, 5>([&](auto i) {
    double x = v[i];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) red[i * 16 + wid] = x;
  });
  __syncthreads();
  static_for<0, 5>([&](auto i) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[i * 16 + w];
    v[i] = s;
  });
  __syncthreads();
}

template <typename T, int N, int S_>
__global__ __launch_bounds__(256) void k_finish(const cpx<T>* __restrict__ D, int tg, cpx<T>* __restrict__ scratch,
                                                const T* f_in, T* q, T* f_out, double dt,
                                                double* __restrict__ moments, EpiParams ep) {
  using C = Cfg<T, N, S_>;
  constexpr int P = C::P, K = C::K, Kh = C::Kh, KH1 = C::KH1, Z = C::Z, S = C::S;
  constexpr size_t N3 = size_t(N) * N * N;
  __shared__ double red[5 * 16];
  const int cell = blockIdx.x;
  constexpr size_t DS = size_t(KH1) * K * Z;  // one slab partial
  const cpx<T>* Dc = D + size_t(cell) * tg * S * DS;
  cpx<T>* sc = scratch + size_t(cell) * N3;
  T* Qtmp = reinterpret_cast<T*>(sc + size_t(KH1) * N * N);  // N^3 reals after the spectra
  const int tid = threadIdx.x, nt = blockDim.x;
  constexpr double inv_p3 = 1.0 / (double(P) * P * P);

  // combine the S slab partials for every kept (kx >= 0, ky, kz), then z synthesis
  for (int it = tid; it < KH1 * K; it += nt) {
    const int kx = it / K, ky = it % K;
    cpx<T> a[N];
    static_for<0, N>([&](auto z) { a[z] = cpx<T>{T(0), T(0)}; });
    static_for<0, K>([&](auto kzi) {
      constexpr int kz = decltype(kzi)::value - Kh;
      constexpr int b = ((kz % Z) + Z) % Z;
      cpx<T> acc = {T(0), T(0)};
      static_for<0, S>([&](auto r) {
        const cpx<T> d = Dc[size_t(decltype(r)::value) * DS + size_t(it) * Z + b];
        acc = acc + twiddle<P, -1, long(kz) * decltype(r)::value>(d);
      });
      a[(kz + N) % N] = cpx<T>{T(acc.re * T(inv_p3)), T(acc.im * T(inv_p3))};
    });
    dft<N, +1>(a);
    static_for<0, N>([&](auto z) { sc[(size_t(kx) * N + ky) * N + z] = a[z]; });
  }
  __syncthreads();
  // y synthesis: columns (kx >= 0, z), in place ky -> y
  for (int it = tid; it < KH1 * N; it += nt) {
    const int kx = it / N, z = it % N;
    cpx<T> a[N];
    static_for<0, N>([&](auto y) { a[y] = cpx<T>{T(0), T(0)}; });
    static_for<0, K>([&](auto kyi) {
      a[(decltype(kyi)::value - Kh + N) % N] = sc[(size_t(kx) * N + kyi) * N + z];
    });
    dft<N, +1>(a);
    static_for<0, N>([&](auto y) { sc[(size_t(kx) * N + y) * N + z] = a[y]; });
  }
  __syncthreads();
  // x synthesis (Hermitian in kx) -> real Q; FP64 invariant moments of Q
  double m[5] = {0, 0, 0, 0, 0};
  for (int it = tid; it < N * N; it += nt) {
    const int y = it / N, z = it % N;
    cpx<T> a[N];
    static_for<0, N>([&](auto x) { a[x] = cpx<T>{T(0), T(0)}; });
    static_for<0, KH1>([&](auto kx) {
      const cpx<T> v = sc[(size_t(kx) * N + y) * N + z];
      a[kx] = v;
      if constexpr (decltype(kx)::value > 0) a[N - decltype(kx)::value] = conj(v);
    });
    dft<N, +1>(a);
    const double vy = -ep.L + y * ep.dv, vz = -ep.L + z * ep.dv;
    static_for<0, N>([&](auto x) {
      const T qv = a[x].re;
      Qtmp[(size_t(x) * N + y) * N + z] = qv;
      const double vx = -ep.L + decltype(x)::value * ep.dv;
      const double d = double(qv);
      m[0] += d;
      m[1] += vx * d;
      m[2] += vy * d;
      m[3] += vz * d;
      m[4] += 0.5 * (vx * vx + vy * vy + vz * vz) * d;
    });
  }
  __syncthreads();
  double lam[5] = {0, 0, 0, 0, 0};
  if (ep.conserve) {
    block_reduce5(m, red);
    for (int i = 0; i < 5; ++i) {
      double s = 0.0;
      for (int j = 0; j < 5; ++j) s += ep.minv[i * 5 + j] * m[j];
      lam[i] = s;
    }
  }
  // correct, write Q and/or the Euler update, moments of the result
  const T* fi = f_in ? f_in + size_t(cell) * N3 : nullptr;
  T* qo = q ? q + size_t(cell) * N3 : nullptr;
  T* fo = f_out ? f_out + size_t(cell) * N3 : nullptr;
  double u[5] = {0, 0, 0, 0, 0};
  for (size_t i = tid; i < N3; i += nt) {
    const int x = int(i / (N * N)), y = int((i / N) % N), z = int(i % N);
    const double vx = -ep.L + x * ep.dv, vy = -ep.L + y * ep.dv, vz = -ep.L + z * ep.dv;
    const double e = 0.5 * (vx * vx + vy * vy + vz * vz);
    double qv = double(Qtmp[i]);
    if (ep.conserve) qv -= lam[0] + lam[1] * vx + lam[2] * vy + lam[3] * vz + lam[4] * e;
    if (qo) qo[i] = T(qv);
    if (fo) {
      const T nv = T(double(fi[i]) + dt * qv);
      fo[i] = nv;
      const double d = double(nv);
      u[0] += d;
      u[1] += vx * d;
      u[2] += vy * d;
      u[3] += vz * d;
      u[4] += e * d;
    }
  }
  if (moments && fo) {
    block_reduce5(u, red);
    if (tid == 0) {
      const double w = ep.dv * ep.dv * ep.dv;
      for (int i = 0; i < 5; ++i) moments[size_t(cell) * 5 + i] = u[i] * w;
    }
  }
}

// LDS-resident finish: the kept spectrum (k_x >= 0) of one cell, [k_x][y][z] with the
// z row padded by one, lives in LDS through the z, y and x syntheses; the x pass stores
// its N real outputs in place of the N/2 complex inputs of its own line.
template <typename T, int N>
struct FinLds {
  static constexpr int KH1 = N / 2;
  static constexpr int RS = N + 1;
  static constexpr size_t bytes = size_t(KH1) * N * RS * sizeof(cpx<T>);
  static constexpr bool fits = bytes <= 156 * 1024;
};

template <typename T, int N, int S_>
__global__ __launch_bounds__(512) void k_finish_lds(const cpx<T>* __restrict__ D, int tg, const T* f_in, T* q,
                                                    T* f_out, double dt, double* __restrict__ moments, EpiParams ep) {
  using C = Cfg<T, N, S_>;
  using F = FinLds<T, N>;
  constexpr int P = C::P, K = C::K, Kh = C::Kh, KH1 = C::KH1, Z = C::Z, S = C::S, RS = F::RS;
  static_assert(KH1 == F::KH1, "half spectrum size");
  constexpr size_t N3 = size_t(N) * N * N;
  __shared__ double red[5 * 16];
  extern __shared__ __align__(16) unsigned char lds_raw[];
  cpx<T>* sm = reinterpret_cast<cpx<T>*>(lds_raw);
  const int cell = blockIdx.x;
  constexpr size_t DS = size_t(KH1) * K * Z;  // one slab partial
  const cpx<T>* Dc = D + size_t(cell) * tg * S * DS;
  const int tid = threadIdx.x, nt = blockDim.x;
  constexpr double inv_p3 = 1.0 / (double(P) * P * P);

  // combine the S slab partials for every kept (kx >= 0, ky, kz), then z synthesis; with
  // term groups the cell's partials sit in its first group slot (k_sum_groups)
  for (int it = tid; it < KH1 * K; it += nt) {
    const int kx = it / K, kyi = it % K;
    cpx<T> a[N];
    static_for<0, N>([&](auto z) { a[z] = cpx<T>{T(0), T(0)}; });
    static_for<0, K>([&](auto kzi) {
      constexpr int kz = decltype(kzi)::value - Kh;
      constexpr int b = ((kz % Z) + Z) % Z;
      cpx<T> acc = {T(0), T(0)};
      static_for<0, S>([&](auto r) {
        const cpx<T> d = Dc[size_t(decltype(r)::value) * DS + size_t(it) * Z + b];
        acc = acc + twiddle<P, -1, long(kz) * decltype(r)::value>(d);
      });
      a[(kz + N) % N] = cpx<T>{T(acc.re * T(inv_p3)), T(acc.im * T(inv_p3))};
    });
    dft<N, +1>(a);
    static_for<0, N>([&](auto z) { sm[(size_t(kx) * N + kyi) * RS + z] = a[z]; });
  }
  __syncthreads();
  // y synthesis: columns (kx, z), in place ky -> y
  for (int it = tid; it < KH1 * N; it += nt) {
    const int kx = it / N, z = it % N;
    cpx<T> a[N];
    static_for<0, N>([&](auto y) { a[y] = cpx<T>{T(0), T(0)}; });
    static_for<0, K>([&](auto kyi) {
      a[(decltype(kyi)::value - Kh + N) % N] = sm[(size_t(kx) * N + kyi) * RS + z];
    });
    dft<N, +1>(a);
    static_for<0, N>([&](auto y) { sm[(size_t(kx) * N + y) * RS + z] = a[y]; });
  }
  __syncthreads();
  // x synthesis (Hermitian in kx) -> real Q, stored as pairs (Q[2j], Q[2j+1]) in slot
  // (j, y, z); FP64 invariant moments of Q
  double m[5] = {0, 0, 0, 0, 0};
  for (int it = tid; it < N * N; it += nt) {
    const int y = it / N, z = it % N;
    cpx<T> a[N];
    static_for<0, N>([&](auto x) { a[x] = cpx<T>{T(0), T(0)}; });
    static_for<0, KH1>([&](auto kx) {
      const cpx<T> v = sm[(size_t(decltype(kx)::value) * N + y) * RS + z];
      a[kx] = v;
      if constexpr (decltype(kx)::value > 0) a[N - decltype(kx)::value] = conj(v);
    });
    dft<N, +1>(a);
    const double vy = -ep.L + y * ep.dv, vz = -ep.L + z * ep.dv;
    static_for<0, N>([&](auto x) {
      const double d = double(a[x].re);
      const double vx = -ep.L + decltype(x)::value * ep.dv;
      m[0] += d;
      m[1] += vx * d;
      m[2] += vy * d;
      m[3] += vz * d;
      m[4] += 0.5 * (vx * vx + vy * vy + vz * vz) * d;
    });
    static_for<0, KH1>([&](auto j) {
      constexpr int jj = decltype(j)::value;
      sm[(size_t(jj) * N + y) * RS + z] = cpx<T>{a[2 * jj].re, a[2 * jj + 1].re};
    });
  }
  __syncthreads();
  double lam[5] = {0, 0, 0, 0, 0};
  if (ep.conserve) {
    block_reduce5(m, red);
    for (int i = 0; i < 5; ++i) {
      double sacc = 0.0;
      for (int j = 0; j < 5; ++j) sacc += ep.minv[i * 5 + j] * m[j];
      lam[i] = sacc;
    }
  }
  const T* fi = f_in ? f_in + size_t(cell) * N3 : nullptr;
  T* qo = q ? q + size_t(cell) * N3 : nullptr;
  T* fo = f_out ? f_out + size_t(cell) * N3 : nullptr;
  const T* smr = reinterpret_cast<const T*>(sm);
  double u[5] = {0, 0, 0, 0, 0};
  for (int i = tid; i < int(N3); i += nt) {
    const int x = i / (N * N), y = (i / N) % N, z = i % N;
    const double vx = -ep.L + x * ep.dv, vy = -ep.L + y * ep.dv, vz = -ep.L + z * ep.dv;
    const double e = 0.5 * (vx * vx + vy * vy + vz * vz);
    double qv = double(smr[(((size_t(x >> 1) * N + y) * RS + z) << 1) + (x & 1)]);
    if (ep.conserve) qv -= lam[0] + lam[1] * vx + lam[2] * vy + lam[3] * vz + lam[4] * e;
    if (qo) qo[i] = T(qv);
    if (fo) {
      const T nv = T(double(fi[i]) + dt * qv);
      fo[i] = nv;
      const double d = double(nv);
      u[0] += d;
      u[1] += vx * d;
      u[2] += vy * d;
      u[3] += vz * d;
      u[4] += e * d;
    }
  }
  if (moments && fo) {
    block_reduce5(u, red);
    if (tid == 0) {
      const double w = ep.dv * ep.dv * ep.dv;
      for (int i = 0; i < 5; ++i) moments[size_t(cell) * 5 + i] = u[i] * w;
    }
  }
}

// Finish in two z passes for cells whose kept spectrum exceeds the LDS (FP64 n = 32),
// without the conservation projection (which needs Q's moments before any output):
// pass p combines the slab partials and synthesises along z (keeping the pass's N/2
// planes), then along y and x in LDS, and writes Q, the Euler update and the moments'
// share of its planes.  The slab partials are read once per pass.
template <typename T, int N>
struct FinSplit {
  static constexpr int KH1 = N / 2;
  static constexpr int ZB = N / 2;
  static constexpr int RS = ZB + 1;
  static constexpr size_t bytes = size_t(KH1) * N * RS * sizeof(cpx<T>);
  static constexpr bool fits = bytes <= 156 * 1024;
};

template <typename T, int N, int S_>
__global__ __launch_bounds__(256) void k_finish_split(const cpx<T>* __restrict__ D, int tg, const T* f_in, T* q,
                                                      T* f_out, double dt, double* __restrict__ moments,
                                                      EpiParams ep) {
  using C = Cfg<T, N, S_>;
  using F = FinSplit<T, N>;
  constexpr int P = C::P, K = C::K, Kh = C::Kh, KH1 = C::KH1, Z = C::Z, S = C::S, RS = F::RS, ZB = F::ZB;
  static_assert(KH1 == F::KH1, "half spectrum size");
  constexpr size_t N3 = size_t(N) * N * N;
  __shared__ double red[5 * 16];
  extern __shared__ __align__(16) unsigned char lds_raw[];
  cpx<T>* sm = reinterpret_cast<cpx<T>*>(lds_raw);
  const int cell = blockIdx.x;
  constexpr size_t DS = size_t(KH1) * K * Z;
  const cpx<T>* Dc = D + size_t(cell) * tg * S * DS;
  const int tid = threadIdx.x, nt = blockDim.x;
  constexpr double inv_p3 = 1.0 / (double(P) * P * P);
  const T* fi = f_in ? f_in + size_t(cell) * N3 : nullptr;
  T* qo = q ? q + size_t(cell) * N3 : nullptr;
  T* fo = f_out ? f_out + size_t(cell) * N3 : nullptr;
  double u[5] = {0, 0, 0, 0, 0};
  static_for<0, 2>([&](auto pc) {
    constexpr int z0 = decltype(pc)::value * ZB;
    for (int it = tid; it < KH1 * K; it += nt) {
      const int kx = it / K, kyi = it % K;
      cpx<T> a[N];
      static_for<0, N>([&](auto z) { a[z] = cpx<T>{T(0), T(0)}; });
      static_for<0, K>([&](auto kzi) {
        constexpr int kz = decltype(kzi)::value - Kh;
        constexpr int b = ((kz % Z) + Z) % Z;
        cpx<T> acc = {T(0), T(0)};
        static_for<0, S>([&](auto r) {
          const cpx<T> d = Dc[size_t(decltype(r)::value) * DS + size_t(it) * Z + b];
          acc = acc + twiddle<P, -1, long(kz) * decltype(r)::value>(d);
        });
        a[(kz + N) % N] = cpx<T>{T(acc.re * T(inv_p3)), T(acc.im * T(inv_p3))};
      });
      dft<N, +1>(a);
      static_for<0, ZB>([&](auto zl) { sm[(size_t(kx) * N + kyi) * RS + zl] = a[z0 + decltype(zl)::value]; });
    }
    __syncthreads();
    // y synthesis: columns (kx, z of the pass), in place ky -> y
    for (int it = tid; it < KH1 * ZB; it += nt) {
      const int kx = it / ZB, zl = it % ZB;
      cpx<T> a[N];
      static_for<0, N>([&](auto y) { a[y] = cpx<T>{T(0), T(0)}; });
      static_for<0, K>([&](auto kyi) {
        a[(decltype(kyi)::value - Kh + N) % N] = sm[(size_t(kx) * N + kyi) * RS + zl];
      });
      dft<N, +1>(a);
      static_for<0, N>([&](auto y) { sm[(size_t(kx) * N + y) * RS + zl] = a[y]; });
    }
    __syncthreads();
    // x synthesis (Hermitian in kx) -> real Q of the pass's planes, written out
    for (int it = tid; it < N * ZB; it += nt) {
      const int y = it / ZB, zl = it % ZB, z = z0 + zl;
      cpx<T> a[N];
      static_for<0, N>([&](auto x) { a[x] = cpx<T>{T(0), T(0)}; });
      static_for<0, KH1>([&](auto kx) {
        const cpx<T> v = sm[(size_t(decltype(kx)::value) * N + y) * RS + zl];
        a[kx] = v;
        if constexpr (decltype(kx)::value > 0) a[N - decltype(kx)::value] = conj(v);
      });
      dft<N, +1>(a);
      const double vy = -ep.L + y * ep.dv, vz = -ep.L + z * ep.dv;
      static_for<0, N>([&](auto x) {
        const size_t i = (size_t(decltype(x)::value) * N + y) * N + z;
        const T qv = a[x].re;
        if (qo) qo[i] = qv;
        if (fo) {
          const T nv = T(double(fi[i]) + dt * double(qv));
          fo[i] = nv;
          const double d = double(nv), vx = -ep.L + decltype(x)::value * ep.dv;
          u[0] += d;
          u[1] += vx * d;
          u[2] += vy * d;
          u[3] += vz * d;
          u[4] += 0.5 * (vx * vx + vy * vy + vz * vz) * d;
        }
      });
    }
    __syncthreads();  // the next pass overwrites the LDS
  });
  if (moments && fo) {
    block_reduce5(u, red);
    if (tid == 0) {
      const double w = ep.dv * ep.dv * ep.dv;
      for (int i = 0; i < 5; ++i) moments[size_t(cell) * 5 + i] = u[i] * w;
    }
  }
}

// ------------------------------------------------------------------------------------
// FP64 moments of f: dv^3 sum phi(v) f
template <typename T, int N>
__global__ __launch_bounds__(256) void k_moments(const T* __restrict__ f, double* __restrict__ u_out,
                                                 double L, double dv) {
  constexpr size_t N3 = size_t(N) * N * N;
  __shared__ double red[5 * 16];
  const int cell = blockIdx.x;
  const T* fc = f + size_t(cell) * N3;
  double u[5] = {0, 0, 0, 0, 0};
  for (size_t i = threadIdx.x; i < N3; i += blockDim.x) {
    const int x = int(i / (N * N)), y = int((i / N) % N), z = int(i % N);
    const double vx = -L + x * dv, vy = -L + y * dv, vz = -L + z * dv;
    const double d = double(fc[i]);
    u[0] += d;
    u[1] += vx * d;
    u[2] += vy * d;
    u[3] += vz * d;
    u[4] += 0.5 * (vx * vx + vy * vy + vz * vz) * d;
  }
  block_reduce5(u, red);
  if (threadIdx.x == 0) {
    const double w = dv * dv * dv;
    for (int i = 0; i < 5; ++i) u_out[size_t(cell) * 5 + i] = u[i] * w;
  }
}

// ------------------------------------------------------------------------------------
// term groups: add the partial spectra of groups 1..tg-1 of each cell into group 0
template <typename T>
__global__ __launch_bounds__(256) void k_sum_groups(cpx<T>* __restrict__ D, int tg, int unit_elems) {
  cpx<T>* Dc = D + size_t(blockIdx.y) * tg * unit_elems;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < unit_elems; i += gridDim.x * blockDim.x) {
    cpx<T> acc = Dc[i];
    for (int g = 1; g < tg; ++g) acc = acc + Dc[size_t(g) * unit_elems + i];
    Dc[i] = acc;
  }
}

// ------------------------------------------------------------------------------------
// host launchers

// forward transform of a batch: the LDS-resident kernel where one cell's partial
// spectra fit in LDS, else three passes through the per-cell global scratch
template <typename T, int N>
static hipError_t launch_forward_kernel(const T* f, cpx<T>* fhat, cpx<T>* scr, int cells, hipStream_t st) {
  if constexpr (FwdLds<T, N>::fits) {
    static bool attr_set = false;
    if (!attr_set) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_forward_lds<T, N>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               int(FwdLds<T, N>::bytes));
      if (e != hipSuccess) return e;
      attr_set = true;
    }
    (void)scr;
    constexpr size_t lds = FwdLds<T, N>::bytes;
    hipLaunchKernelGGL((k_forward_lds<T, N>), dim3(cells), dim3(512), lds, st, f, fhat);
  } else if constexpr (FwdSplit<T, N>::fits) {
    static bool attr_set = false;
    if (!attr_set) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_forward_split<T, N>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               int(FwdSplit<T, N>::bytes));
      if (e != hipSuccess) return e;
      attr_set = true;
    }
    (void)scr;
    hipLaunchKernelGGL((k_forward_split<T, N>), dim3(cells), dim3(512), (FwdSplit<T, N>::bytes), st, f, fhat);
  } else {
    hipLaunchKernelGGL((k_forward_f<T, N>), dim3(cells), dim3(256), 0, st, f, fhat, scr);
  }
  return hipGetLastError();
}

template <typename T, int N, int S>
static hipError_t launch_collide_sched(const CollideArgs& a) {
  using C = Cfg<T, N, S>;
  const T* f = static_cast<const T*>(a.f);
  cpx<T>* fhat = static_cast<cpx<T>*>(a.ws_fhat);
  cpx<T>* scr = static_cast<cpx<T>*>(a.ws_scratch);
  cpx<T>* D = static_cast<cpx<T>*>(a.ws_d);
  hipStream_t st = static_cast<hipStream_t>(a.stream);
  const int cells = int(a.n_cells);
  static bool lds_attr_set = false;  // dynamic LDS above 64 KB must be opted into per kernel
  if (!lds_attr_set) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_slab<T, N, S>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, int(C::lds_bytes));
    if (e != hipSuccess) return e;
    lds_attr_set = true;
  }
  prof_mark(kProfForward, true, st);
  const hipError_t ef = launch_forward_kernel<T, N>(f, fhat, scr, cells, st);
  prof_mark(kProfForward, false, st);
  if (ef != hipSuccess) return ef;
  prof_mark(kProfSlab, true, st);
  const int tg = a.term_groups > 1 ? a.term_groups : 1;
  const int xcd = (a.xcd_map && tg == 1 && cells % 8 == 0) ? 1 : 0;
  hipLaunchKernelGGL((k_slab<T, N, S>), dim3(cells * tg * C::S), dim3(C::NT), C::lds_bytes, st, fhat,
                     static_cast<const T*>(a.tables), a.n_terms, D, xcd, tg);
  prof_mark(kProfSlab, false, st);
  prof_mark(kProfFinish, true, st);
  if (tg > 1) {
    constexpr int ue = C::S * C::KH1 * C::K * C::Z;
    hipLaunchKernelGGL((k_sum_groups<T>), dim3((ue + 255) / 256 < 64 ? (ue + 255) / 256 : 64, cells), dim3(256), 0,
                       st, D, tg, ue);
  }
  if constexpr (FinLds<T, N>::fits) {
    static bool fin_attr_set = false;
    if (!fin_attr_set) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_finish_lds<T, N, S>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               int(FinLds<T, N>::bytes));
      if (e != hipSuccess) return e;
      fin_attr_set = true;
    }
    constexpr size_t lds = FinLds<T, N>::bytes;
    hipLaunchKernelGGL((k_finish_lds<T, N, S>), dim3(cells), dim3(512), lds, st, D, tg,
                       static_cast<const T*>(a.f_in), static_cast<T*>(a.q), static_cast<T*>(a.f_out), a.dt,
                       a.moments, a.ep);
  } else {
    bool split = false;
    if constexpr (FinSplit<T, N>::fits) {
      // without the conservation projection the cell's Q can be written plane by plane
      if (!a.ep.conserve) {
        static bool fin_attr_set = false;
        if (!fin_attr_set) {
          const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_finish_split<T, N, S>),
                                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                                   int(FinSplit<T, N>::bytes));
          if (e != hipSuccess) return e;
          fin_attr_set = true;
        }
        hipLaunchKernelGGL((k_finish_split<T, N, S>), dim3(cells), dim3(256), (FinSplit<T, N>::bytes), st, D, tg,
                           static_cast<const T*>(a.f_in), static_cast<T*>(a.q), static_cast<T*>(a.f_out), a.dt,
                           a.moments, a.ep);
        split = true;
      }
    }
    if (!split)
      hipLaunchKernelGGL((k_finish<T, N, S>), dim3(cells), dim3(256), 0, st, D, tg, scr,
                         static_cast<const T*>(a.f_in), static_cast<T*>(a.q), static_cast<T*>(a.f_out), a.dt,
                         a.moments, a.ep);
  }
  prof_mark(kProfFinish, false, st);
  return hipGetLastError();
}

template <typename T, int N>
static hipError_t launch_collide_impl(const CollideArgs& a) {
  using V = Variants<T, N>;
  if (a.variant == 0) return launch_collide_sched<T, N, V::s[0]>(a);
  if constexpr (V::count > 1) {
    if (a.variant == 1) return launch_collide_sched<T, N, V::s[1]>(a);
  }
  return hipErrorInvalidValue;
}

template <typename T, int N>
static hipError_t launch_forward_impl(const void* f, void* fhat, void* scratch, int64_t cells, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  prof_mark(kProfForward, true, st);
  const hipError_t e = launch_forward_kernel<T, N>(static_cast<const T*>(f), static_cast<cpx<T>*>(fhat),
                                                   static_cast<cpx<T>*>(scratch), int(cells), st);
  prof_mark(kProfForward, false, st);
  return e;
}

template <typename T, int N>
static hipError_t launch_moments_impl(const void* f, int64_t cells, double* u, double L, double dv,
                                      void* stream) {
  prof_mark(kProfMoments, true, static_cast<hipStream_t>(stream));
  hipLaunchKernelGGL((k_moments<T, N>), dim3(int(cells)), dim3(256), 0, static_cast<hipStream_t>(stream),
                     static_cast<const T*>(f), u, L, dv);
  prof_mark(kProfMoments, false, static_cast<hipStream_t>(stream));
  return hipGetLastError();
}

template <typename T, int N>
static void sizes_impl(SlabGeometry* g) {
  using Gd = Grid<T, N>;
  using V = Variants<T, N>;
  g->P = Gd::P;
  g->n_variants = V::count;
  for (int i = 0; i < 2; ++i) g->variant_slabs[i] = i < V::count ? V::s[i] : 0;
  g->fhat_elems = size_t(Gd::NRL) * Gd::NPAIR;
  g->table_rows = Gd::NRL;
  g->scratch_elems = size_t(N) * N * N;
  g->npair = Gd::NPAIR;
  g->d_elems = size_t(Gd::KH1) * Gd::K * Gd::P;  // S*KH1*K*Z = KH1*K*P for any S
}

// per-precision dispatch over the compiled velocity grids
template <typename T>
hipError_t launch_collide_t(int n, const CollideArgs& a) {
  switch (n) {
    case 8: return launch_collide_impl<T, 8>(a);
    case 12: return launch_collide_impl<T, 12>(a);
    case 16: return launch_collide_impl<T, 16>(a);
    case 24: return launch_collide_impl<T, 24>(a);
    case 32: return launch_collide_impl<T, 32>(a);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_forward_t(int n, const void* f, void* fhat, void* scratch, int64_t cells, void* stream) {
  switch (n) {
    case 8: return launch_forward_impl<T, 8>(f, fhat, scratch, cells, stream);
    case 12: return launch_forward_impl<T, 12>(f, fhat, scratch, cells, stream);
    case 16: return launch_forward_impl<T, 16>(f, fhat, scratch, cells, stream);
    case 24: return launch_forward_impl<T, 24>(f, fhat, scratch, cells, stream);
    case 32: return launch_forward_impl<T, 32>(f, fhat, scratch, cells, stream);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_moments_t(int n, const void* f, int64_t cells, double* u, double L, double dv, void* stream) {
  switch (n) {
    case 8: return launch_moments_impl<T, 8>(f, cells, u, L, dv, stream);
    case 12: return launch_moments_impl<T, 12>(f, cells, u, L, dv, stream);
    case 16: return launch_moments_impl<T, 16>(f, cells, u, L, dv, stream);
    case 24: return launch_moments_impl<T, 24>(f, cells, u, L, dv, stream);
    case 32: return launch_moments_impl<T, 32>(f, cells, u, L, dv, stream);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
void slab_geometry_t(int n, SlabGeometry* g) {
  switch (n) {
    case 8: sizes_impl<T, 8>(g); return;
    case 12: sizes_impl<T, 12>(g); return;
    case 16: sizes_impl<T, 16>(g); return;
    case 24: sizes_impl<T, 24>(g); return;
    case 32: sizes_impl<T, 32>(g); return;
    default: return;
  }
}

}  // namespace fks
