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
  void* ws_g;
  void* ws_d;
  const void* f_in;  // Euler base (may equal f), or null
  void* q;           // Q output or null
  void* f_out;       // Euler output or null
  double dt;
  double* moments;   // [cells][5] or null
  EpiParams ep;
  void* stream;
};

struct SlabGeometry {
  int P, S, Z;
  size_t fhat_elems;     // complex elements per cell
  size_t scratch_elems;  // complex elements per cell
  size_t g_elems;        // real elements per cell
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

// f = (f + g) / 2 elementwise over n values
hipError_t launch_average(int dtype_is_f32, void* f, const void* g, int64_t n, void* stream);

// transport
struct XportState {
  double* s;    // [nv][3] sub-cell offsets
  int32_t* o;   // [nv][3] cumulative integer shifts
  int32_t* dl;  // [nv][3] shift of the last step
};
hipError_t launch_xport_reset(const XportState& st, int nv, void* stream);
hipError_t launch_xport_advance(const XportState& st, int n, double L, double dt, double dx, void* stream);
hipError_t launch_roll(int dtype_is_f32, const void* fin, void* fout, const int32_t* dl, int nv, int nx,
                       int ny, int nz, void* stream);

}  // namespace fks
