// The collision kernels of Appendix A instantiated for float (one translation unit per
// precision, so that the two compile in parallel).
#include "fks_collide.hpp"

namespace fks {

hipError_t launch_collide_f32(int n, const CollideArgs& a) { return launch_collide_t<float>(n, a); }

hipError_t launch_forward_f32(int n, const void* f, void* fhat, void* scratch, int64_t cells, void* stream) {
  return launch_forward_t<float>(n, f, fhat, scratch, cells, stream);
}

hipError_t launch_moments_f32(int n, const void* f, int64_t cells, double* u, double L, double dv, void* stream) {
  return launch_moments_t<float>(n, f, cells, u, L, dv, stream);
}

void slab_geometry_f32(int n, SlabGeometry* g) { slab_geometry_t<float>(n, g); }

}  // namespace fks
