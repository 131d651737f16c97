// Precision dispatch of the collision kernels (fks_collide.hpp, instantiated in
// fks_collide_f32.hip and fks_collide_f64.hip) and the Heun averaging kernel.
#include <hip/hip_runtime.h>

#include "fks_internal.hpp"

namespace fks {

hipError_t launch_collide_f32(int n, const CollideArgs& a);
hipError_t launch_collide_f64(int n, const CollideArgs& a);
hipError_t launch_forward_f32(int n, const void* f, void* fhat, void* scratch, int64_t cells, void* stream);
hipError_t launch_forward_f64(int n, const void* f, void* fhat, void* scratch, int64_t cells, void* stream);
hipError_t launch_moments_f32(int n, const void* f, int64_t cells, double* u, double L, double dv, void* stream);
hipError_t launch_moments_f64(int n, const void* f, int64_t cells, double* u, double L, double dv, void* stream);
void slab_geometry_f32(int n, SlabGeometry* g);
void slab_geometry_f64(int n, SlabGeometry* g);

// ------------------------------------------------------------------------------------
// Heun combination f = (f + g)/2
template <typename T>
__global__ __launch_bounds__(256) void k_average(T* __restrict__ f, const T* __restrict__ g, int64_t n) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    f[i] = T(0.5) * (f[i] + g[i]);
}

hipError_t launch_average(int dtype_is_f32, void* f, const void* g, int64_t n, void* stream) {
  // at most 2^22 blocks; the threads stride over the rest
  const int64_t blocks = (n + 255) / 256;
  const dim3 grid(unsigned(blocks < (int64_t(1) << 22) ? (blocks > 0 ? blocks : 1) : (int64_t(1) << 22)));
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dtype_is_f32)
    hipLaunchKernelGGL(k_average<float>, grid, dim3(256), 0, st, static_cast<float*>(f),
                       static_cast<const float*>(g), n);
  else
    hipLaunchKernelGGL(k_average<double>, grid, dim3(256), 0, st, static_cast<double*>(f),
                       static_cast<const double*>(g), n);
  return hipGetLastError();
}

bool collide_supported(int n) { return n == 8 || n == 12 || n == 16 || n == 24 || n == 32; }

hipError_t launch_collide(int dtype_is_f32, int n, const CollideArgs& a) {
  return dtype_is_f32 ? launch_collide_f32(n, a) : launch_collide_f64(n, a);
}

hipError_t launch_forward(int dtype_is_f32, int n, const void* f, void* fhat, void* scratch, int64_t cells,
                          void* stream) {
  return dtype_is_f32 ? launch_forward_f32(n, f, fhat, scratch, cells, stream)
                      : launch_forward_f64(n, f, fhat, scratch, cells, stream);
}

hipError_t launch_moments(int dtype_is_f32, int n, const void* f, int64_t cells, double* u, double L,
                          double dv, void* stream) {
  return dtype_is_f32 ? launch_moments_f32(n, f, cells, u, L, dv, stream)
                      : launch_moments_f64(n, f, cells, u, L, dv, stream);
}

void slab_geometry(int dtype_is_f32, int n, SlabGeometry* g) {
  if (dtype_is_f32) slab_geometry_f32(n, g);
  else slab_geometry_f64(n, g);
}

}  // namespace fks
