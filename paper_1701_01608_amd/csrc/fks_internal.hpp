// Internal interfaces between the C ABI host code and the HIP kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace fks {

// Epilogue constants: velocity grid and the inverse Gram matrix (Phi Phi^T)^-1 of the
// collision invariants phi = (1, v_x, v_y, v_z, |v|^2/2) on the grid (FP64).
struct EpiParams {
  double L;
  double dv;
  double minv[25];
  int conserve;
};

struct CollideArgs {
  const void* f;       // input distributions [cells][n^3]
  const void* tables;  // [terms][rows][npair][2] (alpha, alpha') in the plan dtype
  int n_terms;
  int64_t n_cells;
  void* ws_fhat;
  void* ws_scratch;
  void* ws_d;
  const void* f_in;  // Euler base (may equal f), or null
  void* q;           // Q output or null
  void* f_out;       // Euler output or null
  double dt;
  double* moments;   // [cells][5] or null
  EpiParams ep;
  void* stream;
  int variant;  // slab schedule index (SlabGeometry::variant_slabs)
  int xcd_map;  // 1: keep the S slabs of a cell on one XCD
  int term_groups;  // split each slab's term loop over this many workgroups (partials summed)
};

struct SlabGeometry {
  int P;
  int n_variants;        // compiled slab schedules for this (dtype, n)
  int variant_slabs[2];  // slab count S of each schedule
  size_t fhat_elems;     // complex elements per cell
  size_t scratch_elems;  // complex elements per cell
  size_t d_elems;        // complex elements per cell
  int npair;             // half-plane z pencils, (K^2 + 1)/2
  int table_rows;        // k_z rows of fhat and of each table term (k_z = row - n/2)
};

// per-kernel event timing (no-op unless fks_profile_start is active)
enum ProfSlot { kProfForward = 0, kProfSlab = 1, kProfFinish = 2, kProfAdvance = 3, kProfRoll = 4, kProfMoments = 5 };
void prof_mark(int slot, bool begin, hipStream_t stream);

bool collide_supported(int n);
void slab_geometry(int dtype_is_f32, int n, SlabGeometry* g);
hipError_t launch_collide(int dtype_is_f32, int n, const CollideArgs& a);
hipError_t launch_moments(int dtype_is_f32, int n, const void* f, int64_t cells, double* u, double L,
                          double dv, void* stream);

// forward transform of f only (fhat into the workspace layout)
hipError_t launch_forward(int dtype_is_f32, int n, const void* f, void* fhat, void* scratch, int64_t cells,
                          void* stream);

// surrogate kernels
constexpr int kGemmKStep = 64;  // k extent of one GEMM tile step (split-K ranges are multiples)
enum { kEpiF32_ = 0, kEpiBiasSilu_ = 1, kEpiDSilu_ = 2, kEpiBiasBf16_ = 3 };
hipError_t launch_gemm(int a_km, int b_kn, int epi, const void* A, const void* B, int M, int N, int K, int lda,
                       int ldb, const float* bias, float* Cf, void* Ch, const float* Zin, int ldc, void* stream);
hipError_t launch_mse(const float* Y, const float* T, void* dY, int64_t n, double* partial, int blocks, void* stream);
hipError_t launch_sum_partials(const double* partial, int n, double* out, void* stream);
hipError_t launch_transpose_bf16(const void* in, int rows, int cols, void* out, void* stream);
hipError_t launch_colsum(const void* X, int rows, int cols, float* out, float* partial, int max_blocks,
                         void* stream);
hipError_t launch_gemm_dsilu_splitk(const void* A, const void* B, int b_kn, int M, int N, int K, int lda, int ldb,
                                   const float* Zin, void* Ch, int splits, float* partial, void* stream);
hipError_t launch_adam(float* p, float* m, float* v, const float* g, void* p16, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, void* stream);
hipError_t launch_lowmodes(int dtype_is_f32, const void* fhat, int rows, int half, int npair, int K, int Kh, int mh,
                           double box3, void* X, int ldx, float* rho, const double* mom, double L, int64_t cells,
                           void* stream);
// r: the moment-residual indicator per cell (relative; with absolute = 1 times the cell's
// ||q||_2, an absolute error estimate), or null
hipError_t launch_sur_output(const float* Y, int ldy, const float* rho, float scale, int n, double L, float* q, double* r,
                             int absolute, int64_t cells, void* stream);
hipError_t launch_sur_target(const float* q, const float* rho, float inv_scale, float* t, int n3, int64_t cells, void* stream);
hipError_t launch_shift(int n, const float* in, int64_t ld_in, float* out, const double* mom, int sign, double L,
                        const float* rho, float scale, int mode, double* r, int absolute, int64_t cells, void* stream);
hipError_t launch_features(int dtype_is_f32, int n, int modes, const void* f, void* X, int ldx, float* rho,
                           double* mom, int center, double L, int64_t cells, void* stream);
hipError_t launch_compact(const double* r, int cells, double thr, int* list, int* count, void* stream);
hipError_t launch_gather_cells(int scatter, const float* src, float* dst, const int* list, int count, int n3,
                               void* stream);

// Library-owned device scratch of fks_collide_noalloc (one array per device, fixed size):
// its device address on the current device (looked up once per device, then cached).
constexpr size_t kNoAllocScratchBytes = size_t(128) << 20;
hipError_t noalloc_scratch(void** ptr);

// f = (f + g) / 2 elementwise over n values
hipError_t launch_average(int dtype_is_f32, void* f, const void* g, int64_t n, void* stream);

// transport
struct XportState {
  double* s;    // [nv][3] sub-cell offsets
  int32_t* o;   // [nv][3] cumulative integer shifts
  int32_t* dl;  // [nv][3] shift of the last step
  int32_t* d1;  // [3][n] shift pending since f was last moved, per axis and index along it
};
hipError_t launch_clear_pending(int32_t* d1, int n, void* stream);
hipError_t launch_xport_reset(const XportState& st, int n, void* stream);
hipError_t launch_xport_advance(const XportState& st, int n, double L, double dt, double dx, void* stream);
// f_out[j][k] = f_in[(j - delta_k) mod box][k] with the pending shifts of the compact
// table, which it then clears
hipError_t launch_roll(int dtype_is_f32, const void* fin, void* fout, int32_t* d1, int n, double L, int nx,
                       int ny, int nz, void* stream);

// per-cell transport with eq. DM_update / ToPrimitive and optional BGK relaxation
struct StepCellArgs {
  int n;
  double L;
  int nx, ny, nz;
  double* cons;      // [cells][5] conservative variables, updated in place (DM mode)
  double* prim;      // [cells][5] (rho, u, T) out, or null
  double nu;         // BGK collision frequency (scale)
  int nu_density;    // nu_j = nu * rho_j
  double dt;
  void* q;           // BGK: nu (E - f*) out, or null
  double* moments;   // direct moments of the output masses, or null
};
// The shift from fin to fout with eq. DM_update of the conservative variables a.cons from
// fin and this step's shifts (required); mode 0: nothing more; 1: BGK Euler and 2: BGK exact
// relaxation of the shifted masses at the updated U
hipError_t launch_step_cell(int dtype_is_f32, const void* fin, void* fout, int32_t* d1, int mode,
                            const StepCellArgs& a, void* stream);
hipError_t launch_to_primitive(const double* in, double* out, int64_t cells, void* stream);
// normalised non-equilibrium residual (deviatoric stress, heat flux) per cell
hipError_t launch_noneq(int dtype_is_f32, int n, const void* f, int64_t cells, double L, double* r, void* stream);
hipError_t launch_copy(int dtype_is_f32, const void* src, void* dst, int64_t n, void* stream);

}  // namespace fks
