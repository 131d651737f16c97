// C ABI of libfks (declared in include/fks.h): argument validation, FP64 host table
// construction (Appendix A of the paper), workspace layout and launch sequencing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <functional>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <utility>
#include <string>
#include <vector>

#include "fks.h"
#include "fks_internal.hpp"

namespace {

thread_local std::string g_err;

fks_status fail(fks_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

fks_status ok() {
  g_err.clear();
  return FKS_OK;
}

fks_status check_hip(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(FKS_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
  return FKS_OK;
}

bool aligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

constexpr double kPi = 3.14159265358979323846264338327950288;

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_m.
void gauss_legendre(int m, std::vector<double>& x, std::vector<double>& w) {
  x.assign(m, 0.0);
  w.assign(m, 0.0);
  for (int i = 0; i < (m + 1) / 2; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (m + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= m; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (m == 1) p0 = 1.0, p1 = z;
      dp = m * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= m; ++k) {
      const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = m * (z * p1 - p0) / (z * z - 1.0);
    x[i] = -z;
    x[m - 1 - i] = z;
    w[i] = w[m - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// phi_R(s) = int_{-R}^{R} |rho| e^{i rho s} d rho = 2 R^2 [sin(x)/x - 2 sin^2(x/2)/x^2], x = R|s|
double phi_R(double s, double R) {
  const double x = R * std::fabs(s);
  if (x < 1e-4) return R * R * (1.0 - x * x / 4.0);
  const double h = std::sin(0.5 * x);
  return 2.0 * R * R * (std::sin(x) / x - 2.0 * h * h / (x * x));
}

// psi_R(s) = int over the radius-R disc of e^{i eta.y}, |eta| = s = 2 pi R^2 J1(x)/x, x = R s
double psi_R(double s, double R) {
  const double x = R * std::fabs(s);
  if (x < 1e-5) return 2.0 * kPi * R * R * (0.5 - x * x / 16.0);
  return 2.0 * kPi * R * R * ::j1(x) / x;
}

}  // namespace

namespace fks {
namespace {
struct ProfState {
  bool on = false;
  struct Rec {
    int slot;
    hipEvent_t b, e;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  int open_slot = -1;
  hipEvent_t open_ev = nullptr;
  hipError_t err = hipSuccess;
};
ProfState g_prof;

hipEvent_t prof_event() {
  if (!g_prof.pool.empty()) {
    hipEvent_t e = g_prof.pool.back();
    g_prof.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  const hipError_t r = hipEventCreate(&e);
  if (r != hipSuccess && g_prof.err == hipSuccess) g_prof.err = r;
  return e;
}
}  // namespace

void prof_mark(int slot, bool begin, hipStream_t stream) {
  if (!g_prof.on) return;
  hipEvent_t e = prof_event();
  if (!e) return;
  const hipError_t r = hipEventRecord(e, stream);
  if (r != hipSuccess && g_prof.err == hipSuccess) g_prof.err = r;
  if (begin) {
    g_prof.open_slot = slot;
    g_prof.open_ev = e;
  } else if (g_prof.open_slot == slot && g_prof.open_ev) {
    g_prof.recs.push_back({slot, g_prof.open_ev, e});
    g_prof.open_ev = nullptr;
    g_prof.open_slot = -1;
  } else {
    g_prof.pool.push_back(e);
  }
}
}  // namespace fks

struct fks_plan_s {
  fks_collide_desc d{};
  int64_t max_cells = 0;
  int n = 0, K = 0, Kh = 0;
  int n_terms = 0;  // including the loss term
  size_t esize = 0;
  fks::SlabGeometry geo{};
  std::vector<unsigned char> host_tables;  // [terms][K^3][2] in the plan dtype
  fks::EpiParams ep{};
  void* d_tables = nullptr;
  void* d_ws = nullptr;
  size_t ws_bytes = 0;
  bool bound = false;
  // workspace carve-up (byte offsets)
  size_t off_fhat = 0, off_scr = 0, off_d = 0;
  // slab schedule (index into geo.variant_slabs) and workgroup-to-XCD mapping
  int variant = 0;
  int xcd_map = 1;
  // term groups: each slab's term loop split over tg workgroups (latency of small
  // batches); the workspace holds partials for up to tg_max groups
  int tg = 1, tg_max = 1;
};

// Surrogate: FP32 master parameters, Adam moments, gradients and BF16 weight copies in
// the caller's parameter buffer; activations in the caller's workspace.
struct fks_sur_s {
  int n = 0, modes = 0, width = 0;
  float scale = 1.0f;  // Q = scale * rho^2 * y
  bool center = false; // network works in each cell's mean-velocity frame
  int64_t max_batch = 0;
  int fin = 0, fout = 0;  // features 2*modes^3, outputs n^3
  size_t n_params = 0;
  size_t off_w[3] = {}, off_b[3] = {};  // element offsets into one FP32 tensor
  void* d_params = nullptr;
  void* d_ws = nullptr;
  size_t param_bytes = 0, ws_bytes = 0;
  // parameter buffer carve-up (bytes)
  size_t p_master = 0, p_m = 0, p_v = 0, p_g = 0, p_w16 = 0;
  // workspace carve-up (bytes)
  size_t w_z1 = 0, w_z2 = 0, w_h1 = 0, w_h2 = 0, w_y = 0, w_dy = 0, w_dz1 = 0, w_dz2 = 0, w_part = 0, w_rho = 0,
         w_r = 0, w_list = 0, w_cnt = 0, w_x = 0, w_gf = 0, w_gq = 0, w_cs = 0, w_sk = 0, w_mom = 0, w_ta = 0,
         w_tb = 0, w_w3t = 0;
  int part_blocks = 1024;
  int splits = 1;  // split K of the output layer's input gradient (K = n^3)
  int64_t adam_t = 0;
  bool bound = false;
};

struct fks_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

struct fks_xport_s {
  int n = 0, nx = 0, ny = 0, nz = 0;
  double L = 0.0, dx = 0.0;
  void* d_state = nullptr;
  bool bound = false;
};

namespace {

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }
constexpr int64_t kSmallBatch = 32;   // plans up to this many cells get term-group workspace
constexpr int kMaxTermGroups = 32;

// Separable terms in FP64: for every direction e_t (and radial node) the pair
// (alpha_t(k), alpha'_t(k)) over the kept modes; the loss term (-1, lambda(k)) last.
void build_tables(fks_plan_s* p, std::vector<double>& A, std::vector<double>& Ap) {
  const fks_collide_desc& d = p->d;
  const int K = p->K, Kh = p->Kh;
  const size_t K3 = size_t(K) * K * K;
  const double R = d.R;
  std::vector<double> xi(K);
  for (int i = 0; i < K; ++i) xi[i] = kPi * (i - Kh) / d.L;
  struct Dir {
    double e[3], w;
  };
  std::vector<Dir> dirs;
  for (int pp = 0; pp < d.a1; ++pp)
    for (int q = 0; q < d.a2; ++q) {
      const double th = (pp + 0.5) * kPi / d.a1, ph = q * kPi / d.a2;
      dirs.push_back({{std::sin(th) * std::cos(ph), std::sin(th) * std::sin(ph), std::cos(th)},
                      kPi * kPi * std::sin(th) / (double(d.a1) * d.a2)});
    }
  const bool hs = d.kernel == FKS_HARD_SPHERES;
  const int nr = hs ? 1 : d.n_radial;
  std::vector<double> rho(nr), wrho(nr);
  if (!hs) {
    std::vector<double> gx, gw;
    gauss_legendre(nr, gx, gw);
    for (int r = 0; r < nr; ++r) {
      rho[r] = 0.5 * R * (gx[r] + 1.0);
      wrho[r] = 0.5 * R * gw[r];
    }
  }
  // disc integral in |y| for the power-law kernel: two Gauss-Legendre panels per radial node
  const int ng = 64;
  std::vector<double> gx, gw;
  gauss_legendre(ng, gx, gw);
  const int n_dir_terms = int(dirs.size()) * nr;
  p->n_terms = n_dir_terms + 1;
  A.assign(size_t(p->n_terms) * K3, 0.0);
  Ap.assign(size_t(p->n_terms) * K3, 0.0);
  std::vector<double> yn, yw;  // per radial node: panel nodes and weights incl. 2 pi y' B~
  for (size_t t = 0; t < dirs.size(); ++t) {
    const Dir& D = dirs[t];
    for (int r = 0; r < nr; ++r) {
      const size_t term = t * nr + r;
      double* a = &A[term * K3];
      double* b = &Ap[term * K3];
      if (!hs) {
        yn.clear();
        yw.clear();
        const double split = std::fmin(R, 8.0 * rho[r]);
        const double lo[2] = {0.0, split}, hi[2] = {split, R};
        for (int pnl = 0; pnl < 2; ++pnl) {
          if (hi[pnl] <= lo[pnl]) continue;
          for (int i = 0; i < ng; ++i) {
            const double y = lo[pnl] + 0.5 * (hi[pnl] - lo[pnl]) * (gx[i] + 1.0);
            const double wy = 0.5 * (hi[pnl] - lo[pnl]) * gw[i];
            const double bt = 4.0 * d.C * std::pow(rho[r] * rho[r] + y * y, 0.5 * (d.alpha - 1.0));
            yn.push_back(y);
            yw.push_back(2.0 * kPi * y * bt * wy);
          }
        }
      }
      for (int i = 0; i < K; ++i)
        for (int j = 0; j < K; ++j)
          for (int l = 0; l < K; ++l) {
            const double x0 = xi[i], x1 = xi[j], x2 = xi[l];
            const double pr = x0 * D.e[0] + x1 * D.e[1] + x2 * D.e[2];
            const double q0 = x0 - pr * D.e[0], q1 = x1 - pr * D.e[1], q2 = x2 - pr * D.e[2];
            const double sp = std::sqrt(q0 * q0 + q1 * q1 + q2 * q2);
            const size_t m = (size_t(i) * K + j) * K + l;
            if (hs) {
              a[m] = phi_R(pr, R);
              b[m] = D.w * 4.0 * d.C * psi_R(sp, R);
            } else {
              a[m] = 2.0 * wrho[r] * rho[r] * std::cos(rho[r] * pr);
              double g = 0.0;
              for (size_t u = 0; u < yn.size(); ++u) g += yw[u] * ::j0(yn[u] * sp);
              b[m] = D.w * g;
            }
          }
    }
  }
  // loss term: B_F(m, m) by the same quadrature, with the sign of the loss
  double* al = &A[size_t(n_dir_terms) * K3];
  double* bl = &Ap[size_t(n_dir_terms) * K3];
  for (size_t m = 0; m < K3; ++m) {
    double lam = 0.0;
    for (int t = 0; t < n_dir_terms; ++t) lam += A[size_t(t) * K3 + m] * Ap[size_t(t) * K3 + m];
    al[m] = -1.0;
    bl[m] = lam;
  }
  // Balance the two factors of every term: (alpha, alpha') -> (s alpha, alpha'/s) leaves
  // the product, hence Q, unchanged.  Both factors share one complex transform (real
  // and imaginary part), so their rounding errors mix; with the loss weight lambda four
  // orders of magnitude above 1 the small factor would lose that many digits.  s makes
  // the two factors equally large on the spectrum of a temperature-2 Maxwellian,
  // weight exp(-|xi|^2).
  for (int t = 0; t < p->n_terms; ++t) {
    double sa = 0.0, sb = 0.0;
    for (int i = 0; i < K; ++i)
      for (int j = 0; j < K; ++j)
        for (int l = 0; l < K; ++l) {
          const size_t m = (size_t(i) * K + j) * K + l;
          const double w = std::exp(-(xi[i] * xi[i] + xi[j] * xi[j] + xi[l] * xi[l]));
          sa += w * A[size_t(t) * K3 + m] * A[size_t(t) * K3 + m];
          sb += w * Ap[size_t(t) * K3 + m] * Ap[size_t(t) * K3 + m];
        }
    if (!(sa > 0.0) || !(sb > 0.0)) continue;
    const double sc = std::pow(sb / sa, 0.25);
    for (size_t m = 0; m < K3; ++m) {
      A[size_t(t) * K3 + m] *= sc;
      Ap[size_t(t) * K3 + m] /= sc;
    }
  }
}

// (Phi Phi^T)^-1 for phi = (1, v_x, v_y, v_z, |v|^2/2) over the velocity grid.
bool build_projection(fks_plan_s* p) {
  const int n = p->n;
  const double L = p->d.L, dv = 2.0 * L / n;
  double G[5][10] = {};
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int k = 0; k < n; ++k) {
        const double v[3] = {-L + i * dv, -L + j * dv, -L + k * dv};
        const double ph[5] = {1.0, v[0], v[1], v[2], 0.5 * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2])};
        for (int a = 0; a < 5; ++a)
          for (int b = 0; b < 5; ++b) G[a][b] += ph[a] * ph[b];
      }
  for (int a = 0; a < 5; ++a) G[a][5 + a] = 1.0;
  for (int c = 0; c < 5; ++c) {  // Gauss-Jordan with partial pivoting
    int piv = c;
    for (int r = c + 1; r < 5; ++r)
      if (std::fabs(G[r][c]) > std::fabs(G[piv][c])) piv = r;
    if (std::fabs(G[piv][c]) < 1e-300) return false;
    if (piv != c)
      for (int k = 0; k < 10; ++k) std::swap(G[c][k], G[piv][k]);
    const double inv = 1.0 / G[c][c];
    for (int k = 0; k < 10; ++k) G[c][k] *= inv;
    for (int r = 0; r < 5; ++r)
      if (r != c) {
        const double fct = G[r][c];
        for (int k = 0; k < 10; ++k) G[r][k] -= fct * G[c][k];
      }
  }
  for (int a = 0; a < 5; ++a)
    for (int b = 0; b < 5; ++b) p->ep.minv[a * 5 + b] = G[a][5 + b];
  p->ep.L = L;
  p->ep.dv = dv;
  p->ep.conserve = (p->d.flags & FKS_CONSERVE) ? 1 : 0;
  return true;
}

fks_status check_plan_ready(const fks_plan_s* p) {
  if (!p) return fail(FKS_E_ARG, "null plan");
  if (!p->bound) return fail(FKS_E_STATE, "plan buffers not bound (call fks_plan_bind)");
  return FKS_OK;
}

// Q / Euler over n_cells cells in chunks of max_cells.
// groups actually used for tg requested: ceil(terms / ceil(terms / tg)), so none is empty
int effective_groups(int n_terms, int tg) {
  if (tg <= 1) return 1;
  const int tpg = (n_terms + tg - 1) / tg;
  return (n_terms + tpg - 1) / tpg;
}

// Workspace regions of one chunk of `cells` cells: fhat, the forward/finish scratch, slab
// partials (for the plan's term groups).
struct WsLayout {
  size_t off_fhat, off_scr, off_d, bytes;
};
WsLayout ws_layout(const fks_plan_s* p, int64_t cells, int groups) {
  const size_t cs = p->esize * 2;  // complex element
  WsLayout w{};
  size_t off = 0;
  w.off_fhat = off;
  off = round256(off + size_t(cells) * p->geo.fhat_elems * cs);
  w.off_scr = off;
  off = round256(off + size_t(cells) * p->geo.scratch_elems * cs);
  w.off_d = off;
  off = round256(off + size_t(cells) * groups * p->geo.d_elems * cs);
  w.bytes = off;
  return w;
}

fks_status run_collide_in(fks_plan_s* p, void* ws_base, const WsLayout& w, int64_t chunk, const void* f,
                          const void* f_in, void* q, void* f_out, double dt, int64_t n_cells, double* moments,
                          void* stream) {
  const size_t cell_bytes = size_t(p->n) * p->n * p->n * p->esize;
  const int f32 = p->d.dtype == FKS_F32;
  for (int64_t c0 = 0; c0 < n_cells; c0 += chunk) {
    const int64_t c = (n_cells - c0 < chunk) ? (n_cells - c0) : chunk;
    fks::CollideArgs a{};
    a.f = static_cast<const unsigned char*>(f) + size_t(c0) * cell_bytes;
    a.tables = p->d_tables;
    a.n_terms = p->n_terms;
    a.n_cells = c;
    unsigned char* ws = static_cast<unsigned char*>(ws_base);
    a.ws_fhat = ws + w.off_fhat;
    a.ws_scratch = ws + w.off_scr;
    a.ws_d = ws + w.off_d;
    a.f_in = f_in ? static_cast<const unsigned char*>(f_in) + size_t(c0) * cell_bytes : nullptr;
    a.q = q ? static_cast<unsigned char*>(q) + size_t(c0) * cell_bytes : nullptr;
    a.f_out = f_out ? static_cast<unsigned char*>(f_out) + size_t(c0) * cell_bytes : nullptr;
    a.dt = dt;
    a.moments = moments ? moments + size_t(c0) * 5 : nullptr;
    a.ep = p->ep;
    a.stream = stream;
    a.variant = p->variant;
    a.xcd_map = p->xcd_map;
    a.term_groups = effective_groups(p->n_terms, p->tg);
    const fks_status s = check_hip(fks::launch_collide(f32, p->n, a), "collide launch");
    if (s != FKS_OK) return s;
  }
  return ok();
}

// Q / Euler over n_cells cells in chunks of max_cells through the plan's bound workspace.
fks_status run_collide(fks_plan_s* p, const void* f, const void* f_in, void* q, void* f_out, double dt,
                       int64_t n_cells, double* moments, void* stream) {
  if (!p->d_ws) return fail(FKS_E_STATE, "plan workspace not bound (fks_plan_bind with a workspace)");
  const WsLayout w{p->off_fhat, p->off_scr, p->off_d, p->ws_bytes};
  return run_collide_in(p, p->d_ws, w, p->max_cells, f, f_in, q, f_out, dt, n_cells, moments, stream);
}

bool ranges_overlap(const void* a, const void* b, size_t bytes) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return x < y + bytes && y < x + bytes;
}

}  // namespace

extern "C" {

const char* fks_last_error(void) { return g_err.c_str(); }

fks_status fks_profile_start(void) {
  fks::g_prof.on = true;
  fks::g_prof.err = hipSuccess;
  return ok();
}

fks_status fks_profile_stop(fks_profile_stats* out) {
  if (!out) return fail(FKS_E_ARG, "null argument");
  std::memset(out, 0, sizeof(*out));
  auto& P = fks::g_prof;
  P.on = false;
  fks_status st = FKS_OK;
  for (auto& r : P.recs) {
    if (st == FKS_OK) {
      float ms = 0.f;
      hipError_t e = hipEventSynchronize(r.e);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.b, r.e);
      if (e != hipSuccess) {
        st = fail(FKS_E_DEVICE, "profile events: %s", hipGetErrorString(e));
      } else if (r.slot >= 0 && r.slot < 8) {
        out->total_ms[r.slot] += ms;
        out->launches[r.slot] += 1;
      }
    }
    P.pool.push_back(r.b);
    P.pool.push_back(r.e);
  }
  P.recs.clear();
  if (st == FKS_OK && P.err != hipSuccess) st = fail(FKS_E_DEVICE, "profile: %s", hipGetErrorString(P.err));
  return st == FKS_OK ? ok() : st;
}
const char* fks_version(void) { return "fks 0.1 (gfx950)"; }

constexpr int64_t kMaxChunkCells = int64_t(1) << 19;

fks_status fks_plan_create(const fks_collide_desc* desc, int64_t max_cells, fks_plan* out) {
  if (!desc || !out) return fail(FKS_E_ARG, "null argument");
  *out = nullptr;
  const fks_collide_desc& d = *desc;
  if (d.n < 4 || d.n % 2) return fail(FKS_E_ARG, "n must be even and >= 4 (got %d)", d.n);
  if (!fks::collide_supported(d.n)) return fail(FKS_E_UNSUPPORTED, "n = %d has no compiled kernels", d.n);
  if (!(d.L > 0.0) || !std::isfinite(d.L)) return fail(FKS_E_ARG, "L must be positive");
  if (!(d.R > 0.0) || !std::isfinite(d.R)) return fail(FKS_E_ARG, "R must be positive");
  if (!(d.flags & FKS_ALLOW_OVERLAP) && d.R > 4.0 * d.L / (3.0 + std::sqrt(2.0)) * (1.0 + 1e-12))
    return fail(FKS_E_ARG, "R = %g exceeds the no-overlap bound 4L/(3+sqrt 2) = %g", d.R,
                4.0 * d.L / (3.0 + std::sqrt(2.0)));
  if (!(d.C > 0.0) || !std::isfinite(d.C)) return fail(FKS_E_ARG, "C must be positive");
  if (d.a1 < 1 || d.a1 > 64 || d.a2 < 1 || d.a2 > 64) return fail(FKS_E_ARG, "a1, a2 must be in [1, 64]");
  if (d.kernel != FKS_HARD_SPHERES && d.kernel != FKS_VHS) return fail(FKS_E_ARG, "unknown kernel %d", d.kernel);
  if (d.kernel == FKS_VHS) {
    if (d.n_radial < 1 || d.n_radial > 64) return fail(FKS_E_ARG, "n_radial must be in [1, 64]");
    if (!(d.alpha >= 0.0 && d.alpha < 1.0)) return fail(FKS_E_ARG, "VHS alpha must be in [0, 1)");
  }
  if (d.dtype != FKS_F32 && d.dtype != FKS_F64) return fail(FKS_E_ARG, "dtype must be FKS_F32 or FKS_F64");
  if (d.flags & ~(FKS_CONSERVE | FKS_ALLOW_OVERLAP)) return fail(FKS_E_ARG, "unknown flags 0x%x", d.flags);
  // one chunk's slab launch (cells x slabs x threads per slab, at most 4608 threads per
  // cell) stays below the 2^32 threads of a grid
  if (max_cells < 1 || max_cells > kMaxChunkCells)
    return fail(FKS_E_ARG, "max_cells out of range (1 .. %lld)", (long long)kMaxChunkCells);
  const int nr = d.kernel == FKS_VHS ? d.n_radial : 1;
  if (int64_t(d.a1) * d.a2 * nr > 8192) return fail(FKS_E_ARG, "too many separable terms");

  fks_plan_s* p = new (std::nothrow) fks_plan_s();
  if (!p) return fail(FKS_E_ARG, "out of host memory");
  p->d = d;
  p->max_cells = max_cells;
  p->n = d.n;
  p->K = d.n - 1;
  p->Kh = d.n / 2 - 1;
  p->esize = d.dtype == FKS_F32 ? 4 : 8;
  fks::slab_geometry(d.dtype == FKS_F32, d.n, &p->geo);
  // the kernels address one table term block and one cell's fhat with 32-bit offsets
  const double tab_bytes = double(int64_t(d.a1) * d.a2 * nr + 1) * p->geo.table_rows * p->geo.npair * 2 * p->esize;
  if (tab_bytes >= 2147483648.0) {
    delete p;
    return fail(FKS_E_ARG, "kernel tables would exceed 2 GiB; use fewer directions or radial nodes");
  }
  std::vector<double> A, Ap;
  build_tables(p, A, Ap);
  // device layout [term][kz][half-plane pencil][2]: the kernels read the mirror pencil's
  // values through the evenness alpha(-k) = alpha(k)
  const int K = p->K, Kh = p->Kh, npair = p->geo.npair, rows = p->geo.table_rows;
  const size_t K3 = size_t(K) * K * K;
  // rows k_z = row - n/2: row 0 (Nyquist) and rows >= n stay zero
  p->host_tables.assign(size_t(p->n_terms) * rows * npair * 2 * p->esize, 0);
  for (size_t t = 0; t < size_t(p->n_terms); ++t)
    for (int kzi = 0; kzi < K; ++kzi)
      for (int pp = 0; pp < npair; ++pp) {
        int kx, ky;
        if (pp < Kh * K) {
          kx = 1 + pp / K;
          ky = pp % K - Kh;
        } else {
          kx = 0;
          ky = pp - Kh * K;
        }
        const size_t m = (size_t(kx + Kh) * K + (ky + Kh)) * K + kzi;
        const size_t i = ((t * rows + kzi + 1) * npair + pp) * 2;
        if (d.dtype == FKS_F32) {
          float* h = reinterpret_cast<float*>(p->host_tables.data());
          h[i] = float(A[t * K3 + m]);
          h[i + 1] = float(Ap[t * K3 + m]);
        } else {
          double* h = reinterpret_cast<double*>(p->host_tables.data());
          h[i] = A[t * K3 + m];
          h[i + 1] = Ap[t * K3 + m];
        }
      }
  if (!build_projection(p)) {
    delete p;
    return fail(FKS_E_ARG, "singular invariant Gram matrix");
  }
  p->tg_max = (max_cells <= kSmallBatch) ? (p->n_terms < kMaxTermGroups ? p->n_terms : kMaxTermGroups) : 1;
  const WsLayout w = ws_layout(p, max_cells, p->tg_max);
  p->off_fhat = w.off_fhat;
  p->off_scr = w.off_scr;
  p->off_d = w.off_d;
  p->ws_bytes = w.bytes;
  *out = p;
  return ok();
}

fks_status fks_plan_sizes(fks_plan p, size_t* table_bytes, size_t* workspace_bytes) {
  if (!p || !table_bytes || !workspace_bytes) return fail(FKS_E_ARG, "null argument");
  *table_bytes = p->host_tables.size();
  *workspace_bytes = p->ws_bytes;
  return ok();
}

fks_status fks_plan_info(fks_plan p, int32_t* n_terms, int32_t* pad) {
  if (!p || !n_terms || !pad) return fail(FKS_E_ARG, "null argument");
  *n_terms = p->n_terms;
  *pad = p->geo.P;
  return ok();
}

// Side streams for concurrent groups, per device, created once and kept until the process
// ends (default priority, non-blocking), with one fork event and one join event per side
// stream (timing disabled).
namespace {
constexpr int kMaxSide = 7;
struct SidePool {
  std::mutex use;  // one fork/join at a time per device (the events are shared)
  bool ready = false;
  hipStream_t s[kMaxSide] = {};
  hipEvent_t fork = nullptr, join[kMaxSide] = {};
};
std::mutex g_side_mu;
SidePool g_side[64];

// Creates the current device's side streams (idempotent); false if they cannot be made.
bool side_pool_init(SidePool** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return false;
  std::lock_guard<std::mutex> lk(g_side_mu);
  SidePool& sp = g_side[dev];
  if (!sp.ready) {
    if (hipEventCreateWithFlags(&sp.fork, hipEventDisableTiming) != hipSuccess) return false;
    for (int i = 0; i < kMaxSide; ++i) {
      if (hipStreamCreateWithFlags(&sp.s[i], hipStreamNonBlocking) != hipSuccess) return false;
      if (hipEventCreateWithFlags(&sp.join[i], hipEventDisableTiming) != hipSuccess) return false;
    }
    sp.ready = true;
  }
  *out = &sp;
  return true;
}
}  // namespace

fks_status fks_plan_bind(fks_plan p, void* d_tables, size_t table_bytes, void* d_workspace, size_t workspace_bytes,
                         void* stream) {
  if (!p || !d_tables) return fail(FKS_E_ARG, "null argument");
  if (!d_workspace && workspace_bytes != 0) return fail(FKS_E_ARG, "null workspace with a nonzero size");
  if (!aligned(d_tables) || (d_workspace && !aligned(d_workspace)))
    return fail(FKS_E_ARG, "buffers must be 256-byte aligned");
  if (table_bytes < p->host_tables.size())
    return fail(FKS_E_WORKSPACE, "table buffer %zu < %zu bytes", table_bytes, p->host_tables.size());
  if (d_workspace && workspace_bytes < p->ws_bytes)
    return fail(FKS_E_WORKSPACE, "workspace %zu < %zu bytes", workspace_bytes, p->ws_bytes);
  fks_status s = check_hip(hipMemcpyAsync(d_tables, p->host_tables.data(), p->host_tables.size(),
                                          hipMemcpyHostToDevice, static_cast<hipStream_t>(stream)),
                           "table upload");
  if (s != FKS_OK) return s;
  // the host copy stays alive in the plan until destroy; make the upload complete
  // before returning so that a caller may free its stream right after binding
  s = check_hip(hipStreamSynchronize(static_cast<hipStream_t>(stream)), "table upload sync");
  if (s != FKS_OK) return s;
  p->d_tables = d_tables;
  p->d_ws = d_workspace;
  p->bound = true;
  // the side streams of concurrent grouped calls, made here (outside any stream capture);
  // without them grouped calls run their groups one after another
  SidePool* sp = nullptr;
  (void)side_pool_init(&sp);
  return ok();
}

fks_status fks_collide(fks_plan p, const void* f, void* q, int64_t n_cells, void* stream) {
  fks_status s = check_plan_ready(p);
  if (s != FKS_OK) return s;
  if (n_cells < 0) return fail(FKS_E_ARG, "n_cells < 0");
  if (n_cells == 0) return ok();
  if (!f || !q) return fail(FKS_E_ARG, "null f or q");
  const size_t bytes = size_t(n_cells) * p->n * p->n * p->n * p->esize;
  if (ranges_overlap(f, q, bytes)) return fail(FKS_E_ARG, "q must not overlap f");
  return run_collide(p, f, nullptr, q, nullptr, 0.0, n_cells, nullptr, stream);
}

fks_status fks_collide_noalloc(fks_plan p, const void* f, void* q, int64_t n_cells, void* stream) {
  if (!p) return fail(FKS_E_ARG, "null plan");
  if (!p->d_tables) return fail(FKS_E_STATE, "plan tables not bound (call fks_plan_bind)");
  if (n_cells < 0) return fail(FKS_E_ARG, "n_cells < 0");
  if (n_cells == 0) return ok();
  if (!f || !q) return fail(FKS_E_ARG, "null f or q");
  const size_t bytes = size_t(n_cells) * p->n * p->n * p->n * p->esize;
  if (ranges_overlap(f, q, bytes)) return fail(FKS_E_ARG, "q must not overlap f");
  const int groups = effective_groups(p->n_terms, p->tg);
  const WsLayout w = ws_layout(p, n_cells, groups);
  if (n_cells > p->max_cells || w.bytes > fks::kNoAllocScratchBytes) {
    // the largest cell count whose layout fits: start from the unrounded per-cell bytes
    const size_t per_cell = (p->geo.fhat_elems + p->geo.scratch_elems + size_t(groups) * p->geo.d_elems) * p->esize * 2;
    int64_t cap = int64_t(fks::kNoAllocScratchBytes / per_cell);
    while (cap > 0 && ws_layout(p, cap, groups).bytes > fks::kNoAllocScratchBytes) --cap;
    while (ws_layout(p, cap + 1, groups).bytes <= fks::kNoAllocScratchBytes) ++cap;
    if (cap > p->max_cells) cap = p->max_cells;
    return fail(FKS_E_ARG, "n_cells = %lld exceeds what the %zu MiB library scratch holds for this plan (%lld cells)",
                static_cast<long long>(n_cells), fks::kNoAllocScratchBytes >> 20, static_cast<long long>(cap));
  }
  void* scratch = nullptr;
  fks_status s = check_hip(fks::noalloc_scratch(&scratch), "library scratch address");
  if (s != FKS_OK) return s;
  return run_collide_in(p, scratch, w, n_cells, f, nullptr, q, nullptr, 0.0, n_cells, nullptr, stream);
}

fks_status fks_relax(fks_plan p, const void* f_in, void* f_out, void* q, double dt, int64_t n_cells,
                     double* d_moments, void* stream) {
  fks_status s = check_plan_ready(p);
  if (s != FKS_OK) return s;
  if (!std::isfinite(dt)) return fail(FKS_E_ARG, "dt must be finite");
  if (n_cells < 0) return fail(FKS_E_ARG, "n_cells < 0");
  if (n_cells == 0) return ok();
  if (!f_in || !f_out) return fail(FKS_E_ARG, "null f_in or f_out");
  const size_t bytes = size_t(n_cells) * p->n * p->n * p->n * p->esize;
  if (f_in != f_out && ranges_overlap(f_in, f_out, bytes)) return fail(FKS_E_ARG, "f_out partially overlaps f_in");
  if (q && (ranges_overlap(q, f_in, bytes) || ranges_overlap(q, f_out, bytes)))
    return fail(FKS_E_ARG, "q must not overlap f_in or f_out");
  return run_collide(p, f_in, f_in, q, f_out, dt, n_cells, d_moments, stream);
}

fks_status fks_moments(fks_plan p, const void* f, int64_t n_cells, double* d_u, void* stream) {
  if (!p) return fail(FKS_E_ARG, "null plan");
  if (n_cells < 0) return fail(FKS_E_ARG, "n_cells < 0");
  if (n_cells == 0) return ok();
  if (!f || !d_u) return fail(FKS_E_ARG, "null f or d_u");
  return check_hip(fks::launch_moments(p->d.dtype == FKS_F32, p->n, f, n_cells, d_u, p->d.L, 2.0 * p->d.L / p->n,
                                       stream),
                   "moments launch") == FKS_OK
             ? ok()
             : FKS_E_DEVICE;
}

fks_status fks_noneq(fks_plan p, const void* f, int64_t n_cells, double* d_r, void* stream) {
  if (!p) return fail(FKS_E_ARG, "null plan");
  if (n_cells < 0) return fail(FKS_E_ARG, "n_cells < 0");
  if (n_cells == 0) return ok();
  if (!f || !d_r) return fail(FKS_E_ARG, "null f or d_r");
  if (n_cells > (int64_t(1) << 31) - 1) return fail(FKS_E_ARG, "too many cells for one call");
  return check_hip(fks::launch_noneq(p->d.dtype == FKS_F32, p->n, f, n_cells, p->d.L, d_r, stream),
                   "non-equilibrium residual") == FKS_OK
             ? ok()
             : FKS_E_DEVICE;
}

fks_status fks_collide_grouped(const fks_plan* plans, int32_t n_groups, const void* const* f, void* const* q,
                               const int64_t* n_cells, void* stream) {
  if (!plans || !f || !q || !n_cells || n_groups < 0) return fail(FKS_E_ARG, "null argument");
  for (int g = 0; g < n_groups; ++g) {
    fks_status s = check_plan_ready(plans[g]);
    if (s != FKS_OK) return s;
    if (n_cells[g] < 0 || (n_cells[g] > 0 && (!f[g] || !q[g])))
      return fail(FKS_E_ARG, "group %d: bad buffers or count", g);
    if (plans[g]->d.dtype != plans[0]->d.dtype) return fail(FKS_E_ARG, "groups must share one dtype");
  }
  // Groups run concurrently, group 0 on the caller's stream and group g > 0 on a side
  // stream forked from it by an event and joined back before the call returns, so the
  // smaller groups fill the CUs the largest leaves idle (its launch tails, its forward and
  // synthesis kernels).  Under stream capture the fork and join become graph edges.  Groups
  // that share a workspace (the same plan twice, or overlapping buffers) run one after
  // another on the caller's stream.
  std::vector<int> active;
  for (int g = 0; g < n_groups; ++g)
    if (n_cells[g] > 0) active.push_back(g);
  bool concurrent = active.size() > 1 && int(active.size()) - 1 <= kMaxSide;
  for (size_t i = 0; concurrent && i < active.size(); ++i)
    for (size_t j = i + 1; j < active.size(); ++j) {
      const fks_plan a = plans[active[i]], b = plans[active[j]];
      const uintptr_t xa = reinterpret_cast<uintptr_t>(a->d_ws), xb = reinterpret_cast<uintptr_t>(b->d_ws);
      if (a == b || (xa < xb + b->ws_bytes && xb < xa + a->ws_bytes)) concurrent = false;
    }
  SidePool* sp = nullptr;
  if (concurrent && !side_pool_init(&sp)) concurrent = false;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!concurrent) {
    for (int g : active) {
      fks_status s = fks_collide(plans[g], f[g], q[g], n_cells[g], stream);
      if (s != FKS_OK) return s;
    }
    return ok();
  }
  std::lock_guard<std::mutex> lk(sp->use);
  fks_status s = check_hip(hipEventRecord(sp->fork, st), "fork event");
  if (s != FKS_OK) return s;
  for (size_t i = 1; i < active.size(); ++i) {
    s = check_hip(hipStreamWaitEvent(sp->s[i - 1], sp->fork, 0), "fork wait");
    if (s != FKS_OK) return s;
  }
  fks_status first_err = FKS_OK;
  for (size_t i = 0; i < active.size(); ++i) {
    const int g = active[i];
    s = fks_collide(plans[g], f[g], q[g], n_cells[g], i == 0 ? stream : static_cast<void*>(sp->s[i - 1]));
    if (s != FKS_OK && first_err == FKS_OK) first_err = s;
  }
  // join every side stream back, also after an error, so no capture is left forked
  for (size_t i = 1; i < active.size(); ++i) {
    s = check_hip(hipEventRecord(sp->join[i - 1], sp->s[i - 1]), "join event");
    if (s == FKS_OK) s = check_hip(hipStreamWaitEvent(st, sp->join[i - 1], 0), "join wait");
    if (s != FKS_OK && first_err == FKS_OK) first_err = s;
  }
  return first_err == FKS_OK ? ok() : first_err;
}

fks_status fks_heun(fks_plan p, void* f, void* f_tmp1, void* f_tmp2, double dt, int32_t n_steps, int64_t n_cells,
                    void* stream) {
  fks_status s = check_plan_ready(p);
  if (s != FKS_OK) return s;
  if (!std::isfinite(dt)) return fail(FKS_E_ARG, "dt must be finite");
  if (n_steps < 0 || n_cells < 0) return fail(FKS_E_ARG, "n_steps and n_cells must be >= 0");
  if (n_steps == 0 || n_cells == 0) return ok();
  if (!f || !f_tmp1 || !f_tmp2) return fail(FKS_E_ARG, "null buffer");
  const size_t bytes = size_t(n_cells) * p->n * p->n * p->n * p->esize;
  if (ranges_overlap(f, f_tmp1, bytes) || ranges_overlap(f, f_tmp2, bytes) || ranges_overlap(f_tmp1, f_tmp2, bytes))
    return fail(FKS_E_ARG, "f, f_tmp1 and f_tmp2 must not overlap");
  const int64_t nval = n_cells * int64_t(p->n) * p->n * p->n;
  for (int st = 0; st < n_steps; ++st) {
    s = run_collide(p, f, f, nullptr, f_tmp1, dt, n_cells, nullptr, stream);
    if (s != FKS_OK) return s;
    s = run_collide(p, f_tmp1, f_tmp1, nullptr, f_tmp2, dt, n_cells, nullptr, stream);
    if (s != FKS_OK) return s;
    s = check_hip(fks::launch_average(p->d.dtype == FKS_F32, f, f_tmp2, nval, stream), "heun average");
    if (s != FKS_OK) return s;
  }
  return ok();
}

void fks_plan_destroy(fks_plan p) { delete p; }

fks_status fks_plan_schedule(fks_plan p, int32_t* slabs, int32_t* xcd_map) {
  if (!p || !slabs || !xcd_map) return fail(FKS_E_ARG, "null argument");
  *slabs = p->geo.variant_slabs[p->variant];
  *xcd_map = p->xcd_map;
  return ok();
}

fks_status fks_plan_set_schedule(fks_plan p, int32_t slabs, int32_t xcd_map) {
  if (!p) return fail(FKS_E_ARG, "null plan");
  for (int v = 0; v < p->geo.n_variants; ++v)
    if (p->geo.variant_slabs[v] == slabs) {
      p->variant = v;
      p->xcd_map = xcd_map ? 1 : 0;
      return ok();
    }
  return fail(FKS_E_UNSUPPORTED, "no compiled schedule with %d slabs for n = %d", slabs, p->n);
}

fks_status fks_plan_set_term_groups(fks_plan p, int32_t tg) {
  if (!p) return fail(FKS_E_ARG, "null plan");
  if (tg < 1) return fail(FKS_E_ARG, "term groups must be >= 1");
  if (tg > p->tg_max)
    return fail(FKS_E_UNSUPPORTED, "at most %d term groups for this plan (small-batch plans only)", p->tg_max);
  p->tg = tg;
  return ok();
}

fks_status fks_plan_get_term_groups(fks_plan p, int32_t* tg, int32_t* tg_max) {
  if (!p || !tg || !tg_max) return fail(FKS_E_ARG, "null argument");
  *tg = effective_groups(p->n_terms, p->tg);
  *tg_max = p->tg_max;
  return ok();
}

namespace {
// Writes the current device's architecture name without feature suffixes ("gfx950") into *out.
void device_name(std::string* out) {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    *out = "unknown";
    return;
  }
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  *out = c == std::string::npos ? a : a.substr(0, c);
}

// cache line: {"device":"gfx950","n":32,"dtype":"f32","terms":17,"cells":4096,"slabs":6,"xcd":1,"ms":15.0}
bool cache_lookup(const char* path, const std::string& key, int* slabs, int* xcd, int* tg) {
  FILE* fp = std::fopen(path, "r");
  if (!fp) return false;
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof(line), fp)) {
    const std::string l(line);
    if (l.find(key) == std::string::npos) continue;
    const size_t ps = l.find("\"slabs\":"), px = l.find("\"xcd\":");
    if (ps == std::string::npos || px == std::string::npos) continue;
    *slabs = std::atoi(l.c_str() + ps + 8);
    *xcd = std::atoi(l.c_str() + px + 6);
    const size_t pt = l.find("\"tg\":");
    *tg = pt == std::string::npos ? 1 : std::atoi(l.c_str() + pt + 5);
    found = true;  // the last matching line wins
  }
  std::fclose(fp);
  return found;
}
}  // namespace

fks_status fks_plan_autotune(fks_plan p, const void* f, void* q, int64_t n_cells, const char* cache_path,
                             void* stream) {
  fks_status s = check_plan_ready(p);
  if (s != FKS_OK) return s;
  if (!f || !q || n_cells < 1) return fail(FKS_E_ARG, "need f, q and n_cells >= 1");
  if (n_cells > p->max_cells) n_cells = p->max_cells;
  std::string dev_name;
  device_name(&dev_name);
  char keybuf[256];
  std::snprintf(keybuf, sizeof(keybuf), "\"device\":\"%s\",\"n\":%d,\"dtype\":\"%s\",\"terms\":%d,\"cells\":%lld",
                dev_name.c_str(), p->n, p->d.dtype == FKS_F32 ? "f32" : "f64", p->n_terms,
                static_cast<long long>(n_cells));
  // the stored line continues with ',"slabs":', so matching the key plus its comma compares the
  // cell count exactly (4096 does not match a line written for 40960)
  const std::string key(keybuf);
  const std::string match = key + ",";
  int cs = 0, cx = 0, ct = 1;
  if (cache_path && cache_lookup(cache_path, match, &cs, &cx, &ct) && fks_plan_set_schedule(p, cs, cx) == FKS_OK &&
      fks_plan_set_term_groups(p, ct) == FKS_OK)
    return ok();
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  s = check_hip(hipEventCreate(&e0), "event");
  if (s != FKS_OK) return s;
  s = check_hip(hipEventCreate(&e1), "event");
  if (s != FKS_OK) {
    (void)hipEventDestroy(e0);
    return s;
  }
  float best = 1e30f;
  int best_v = p->variant, best_x = p->xcd_map, best_t = p->tg;
  for (int v = 0; v < p->geo.n_variants && s == FKS_OK; ++v)
    for (int x = 0; x < 2 && s == FKS_OK; ++x)
      for (int t = 1; t <= p->tg_max && s == FKS_OK; t *= 2) {
        if (x && t > 1) continue;  // the XCD mapping applies to single-group schedules
        p->variant = v;
        p->xcd_map = x;
        p->tg = t;
        s = run_collide(p, f, nullptr, q, nullptr, 0.0, n_cells, nullptr, stream);  // warm-up
        if (s != FKS_OK) break;
        s = check_hip(hipEventRecord(e0, st), "event record");
        for (int r = 0; r < 3 && s == FKS_OK; ++r)
          s = run_collide(p, f, nullptr, q, nullptr, 0.0, n_cells, nullptr, stream);
        if (s == FKS_OK) s = check_hip(hipEventRecord(e1, st), "event record");
        if (s == FKS_OK) s = check_hip(hipEventSynchronize(e1), "event sync");
        float ms = 0.f;
        if (s == FKS_OK) s = check_hip(hipEventElapsedTime(&ms, e0, e1), "elapsed");
        if (s == FKS_OK && ms < best) {
          best = ms;
          best_v = v;
          best_x = x;
          best_t = t;
        }
      }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  p->variant = best_v;
  p->xcd_map = best_x;
  p->tg = best_t;
  if (s != FKS_OK) return s;
  if (cache_path) {
    FILE* fp = std::fopen(cache_path, "a");
    if (fp) {
      std::fprintf(fp, "{%s,\"slabs\":%d,\"xcd\":%d,\"tg\":%d,\"ms\":%.4f}\n", key.c_str(),
                   p->geo.variant_slabs[best_v], best_x, best_t, best / 3.0f);
      std::fclose(fp);
    }
  }
  return ok();
}

// ---- surrogate ----------------------------------------------------------------------
namespace {
unsigned char* B(void* p, size_t off) { return static_cast<unsigned char*>(p) + off; }

// FP32 -> BF16 with round to nearest even (the rounding the device conversion uses)
uint16_t bf16_bits(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return uint16_t((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

constexpr int kColsumBlocks = 32;  // row blocks of the two-pass bias-gradient sums

fks_status sur_ready(const fks_sur_s* s) {
  if (!s) return fail(FKS_E_ARG, "null surrogate");
  if (!s->bound) return fail(FKS_E_STATE, "surrogate buffers not bound (call fks_sur_bind)");
  return FKS_OK;
}

// forward pass of a batch (rows multiple of 128) into Z1, H1, Z2, H2 and Y
// forward pass; the output layer writes y_out ([rows][n^3] FP32) or, if null, the workspace
fks_status sur_forward(fks_sur_s* s, const void* x, int64_t rows, void* stream, float* y_out = nullptr) {
  const float* P = reinterpret_cast<const float*>(B(s->d_params, s->p_master));
  const unsigned char* W16 = B(s->d_params, s->p_w16);
  const int w = s->width, fi = s->fin, fo = s->fout, r = int(rows);
  fks_status st = check_hip(fks::launch_gemm(0, 0, fks::kEpiBiasSilu_, x, W16 + 2 * s->off_w[0], r, w, fi, fi, fi,
                                             P + s->off_b[0], reinterpret_cast<float*>(B(s->d_ws, s->w_z1)),
                                             B(s->d_ws, s->w_h1), nullptr, w, stream),
                            "surrogate layer 1");
  if (st != FKS_OK) return st;
  st = check_hip(fks::launch_gemm(0, 0, fks::kEpiBiasSilu_, B(s->d_ws, s->w_h1), W16 + 2 * s->off_w[1], r, w, w, w, w,
                                  P + s->off_b[1], reinterpret_cast<float*>(B(s->d_ws, s->w_z2)), B(s->d_ws, s->w_h2),
                                  nullptr, w, stream),
                 "surrogate layer 2");
  if (st != FKS_OK) return st;
  return check_hip(fks::launch_gemm(0, 0, fks::kEpiF32_, B(s->d_ws, s->w_h2), W16 + 2 * s->off_w[2], r, fo, w, w, w,
                                    P + s->off_b[2], y_out ? y_out : reinterpret_cast<float*>(B(s->d_ws, s->w_y)),
                                    nullptr, nullptr, fo, stream),
                   "surrogate layer 3");
}

// weight gradient G[M][N] = A^T B for A [r][M], B [r][N] (bf16, batch-major): both are
// transposed to K-contiguous rows first so the GEMM stages its tiles with 16-byte moves
fks_status weight_grad(fks_sur_s* s, const void* A, int M, const void* Bm, int N, int r, float* G, void* stream) {
  void* at = B(s->d_ws, s->w_ta);
  void* bt = B(s->d_ws, s->w_tb);
  fks_status st = check_hip(fks::launch_transpose_bf16(A, r, M, at, stream), "transpose");
  if (st == FKS_OK) st = check_hip(fks::launch_transpose_bf16(Bm, r, N, bt, stream), "transpose");
  if (st == FKS_OK)
    st = check_hip(fks::launch_gemm(0, 0, fks::kEpiF32_, at, bt, M, N, r, r, r, nullptr, G, nullptr, nullptr, N, stream),
                   "weight gradient");
  return st;
}

// gradients of the MSE of the batch against targets t into the gradient buffer
fks_status sur_backward(fks_sur_s* s, const void* x, const float* t, int64_t rows, double* d_loss, void* stream) {
  float* G = reinterpret_cast<float*>(B(s->d_params, s->p_g));
  const unsigned char* W16 = B(s->d_params, s->p_w16);
  const int w = s->width, fi = s->fin, fo = s->fout, r = int(rows);
  void* dy = B(s->d_ws, s->w_dy);
  double* part = reinterpret_cast<double*>(B(s->d_ws, s->w_part));
  fks_status st = check_hip(fks::launch_mse(reinterpret_cast<const float*>(B(s->d_ws, s->w_y)), t, dy,
                                            int64_t(r) * fo, part, s->part_blocks, stream),
                            "surrogate loss");
  if (st != FKS_OK) return st;
  if (d_loss) {
    st = check_hip(fks::launch_sum_partials(part, s->part_blocks, d_loss, stream), "loss sum");
    if (st != FKS_OK) return st;
  }
  // layer 3: dW3 = dY^T H2, db3 = colsum dY, dZ2 = (dY W3) silu'(Z2)
  st = weight_grad(s, dy, fo, B(s->d_ws, s->w_h2), w, r, G + s->off_w[2], stream);
  float* cs = reinterpret_cast<float*>(B(s->d_ws, s->w_cs));
  if (st == FKS_OK) st = check_hip(fks::launch_colsum(dy, r, fo, G + s->off_b[2], cs, kColsumBlocks, stream), "db3");
  // dZ2: K = n^3 is long and M x N = batch x width has few tiles: split K.  Where the
  // large-tile kernel applies, W3 is first transposed to [width][n^3] so that both operands
  // are K-contiguous
  if (st == FKS_OK && r % 256 == 0 && w % 256 == 0) {
    void* w3t = B(s->d_ws, s->w_w3t);
    st = check_hip(fks::launch_transpose_bf16(W16 + 2 * s->off_w[2], fo, w, w3t, stream), "W3 transpose");
    if (st == FKS_OK)
      st = check_hip(fks::launch_gemm_dsilu_splitk(dy, w3t, 0, r, w, fo, fo, fo,
                                                   reinterpret_cast<const float*>(B(s->d_ws, s->w_z2)),
                                                   B(s->d_ws, s->w_dz2), s->splits,
                                                   reinterpret_cast<float*>(B(s->d_ws, s->w_sk)), stream),
                     "dZ2");
  } else if (st == FKS_OK) {
    st = check_hip(fks::launch_gemm_dsilu_splitk(dy, W16 + 2 * s->off_w[2], 1, r, w, fo, fo, w,
                                                 reinterpret_cast<const float*>(B(s->d_ws, s->w_z2)),
                                                 B(s->d_ws, s->w_dz2), s->splits,
                                                 reinterpret_cast<float*>(B(s->d_ws, s->w_sk)), stream),
                   "dZ2");
  }
  // layer 2
  if (st == FKS_OK) st = weight_grad(s, B(s->d_ws, s->w_dz2), w, B(s->d_ws, s->w_h1), w, r, G + s->off_w[1], stream);
  if (st == FKS_OK)
    st = check_hip(fks::launch_colsum(B(s->d_ws, s->w_dz2), r, w, G + s->off_b[1], cs, kColsumBlocks, stream), "db2");
  if (st == FKS_OK)
    st = check_hip(fks::launch_gemm(0, 1, fks::kEpiDSilu_, B(s->d_ws, s->w_dz2), W16 + 2 * s->off_w[1], r, w, w, w, w,
                                    nullptr, nullptr, B(s->d_ws, s->w_dz1),
                                    reinterpret_cast<const float*>(B(s->d_ws, s->w_z1)), w, stream),
                   "dZ1");
  // layer 1
  if (st == FKS_OK) st = weight_grad(s, B(s->d_ws, s->w_dz1), w, x, fi, r, G + s->off_w[0], stream);
  if (st == FKS_OK)
    st = check_hip(fks::launch_colsum(B(s->d_ws, s->w_dz1), r, w, G + s->off_b[0], cs, kColsumBlocks, stream), "db1");
  return st;
}
}  // namespace

fks_status fks_sur_create(int32_t n, int32_t modes, int32_t width, int64_t max_batch, float out_scale, uint32_t flags,
                          fks_sur* out) {
  if (!out) return fail(FKS_E_ARG, "null out");
  *out = nullptr;
  if (flags & ~uint32_t(FKS_SUR_CENTER)) return fail(FKS_E_ARG, "unknown flags");
  if ((flags & FKS_SUR_CENTER) && n != 8 && n != 16 && n != 24 && n != 32)
    return fail(FKS_E_UNSUPPORTED, "centring is built for n = 8, 16, 24, 32");
  if (!(out_scale > 0.0f) || !std::isfinite(out_scale)) return fail(FKS_E_ARG, "out_scale must be positive");
  if (n < 4 || n > 64) return fail(FKS_E_ARG, "n out of range");
  if (modes < 2 || modes % 2 || modes > n - 2) return fail(FKS_E_ARG, "modes must be even and <= n - 2");
  const int64_t fin = 2 * int64_t(modes) * modes * modes, fout = int64_t(n) * n * n;
  if (fin % 128 || fout % 128) return fail(FKS_E_UNSUPPORTED, "2*modes^3 and n^3 must be multiples of 128");
  if (width < 128 || width % 128) return fail(FKS_E_ARG, "width must be a positive multiple of 128");
  if (max_batch < 128 || max_batch % 128 || max_batch > (int64_t(1) << 16))
    return fail(FKS_E_ARG, "max_batch must be a multiple of 128 in [128, 65536]");
  fks_sur_s* s = new (std::nothrow) fks_sur_s();
  if (!s) return fail(FKS_E_ARG, "out of host memory");
  s->n = n;
  s->scale = out_scale;
  s->center = (flags & FKS_SUR_CENTER) != 0;
  s->modes = modes;
  s->width = width;
  s->max_batch = max_batch;
  s->fin = int(fin);
  s->fout = int(fout);
  const size_t w = size_t(width), fi = size_t(fin), fo = size_t(fout);
  size_t o = 0;
  s->off_w[0] = o;  o += w * fi;
  s->off_b[0] = o;  o += w;
  s->off_w[1] = o;  o += w * w;
  s->off_b[1] = o;  o += w;
  s->off_w[2] = o;  o += fo * w;
  s->off_b[2] = o;  o += fo;
  s->n_params = o;
  size_t pb = 0;
  s->p_master = pb;  pb = round256(pb + 4 * o);
  s->p_m = pb;       pb = round256(pb + 4 * o);
  s->p_v = pb;       pb = round256(pb + 4 * o);
  s->p_g = pb;       pb = round256(pb + 4 * o);
  s->p_w16 = pb;     pb = round256(pb + 2 * o);  // same element offsets (biases unused)
  s->param_bytes = pb;
  const size_t Bm = size_t(max_batch);
  size_t wb = 0;
  s->w_z1 = wb;   wb = round256(wb + 4 * Bm * w);
  s->w_z2 = wb;   wb = round256(wb + 4 * Bm * w);
  s->w_h1 = wb;   wb = round256(wb + 2 * Bm * w);
  s->w_h2 = wb;   wb = round256(wb + 2 * Bm * w);
  s->w_y = wb;    wb = round256(wb + 4 * Bm * fo);
  s->w_dy = wb;   wb = round256(wb + 2 * Bm * fo);
  s->w_dz1 = wb;  wb = round256(wb + 2 * Bm * w);
  s->w_dz2 = wb;  wb = round256(wb + 2 * Bm * w);
  s->w_part = wb; wb = round256(wb + 8 * size_t(s->part_blocks));
  s->w_rho = wb;  wb = round256(wb + 4 * Bm);
  s->w_r = wb;    wb = round256(wb + 8 * Bm);
  s->w_list = wb; wb = round256(wb + 4 * Bm);
  s->w_cnt = wb;  wb = round256(wb + 4);
  s->w_x = wb;    wb = round256(wb + 2 * Bm * fi);
  s->w_gf = wb;   wb = round256(wb + 4 * Bm * fo);  // fallback gather buffers (FP32 cells)
  s->w_gq = wb;   wb = round256(wb + 4 * Bm * fo);
  s->w_cs = wb;   wb = round256(wb + 4 * size_t(kColsumBlocks) * (fo > w ? fo : w));
  s->w_mom = wb;  wb = round256(wb + 8 * 5 * Bm);
  // transposed operands of the weight gradients ([features][batch] bf16)
  const size_t tmax = fo > w ? (fo > fi ? fo : fi) : (w > fi ? w : fi);
  s->w_ta = wb;   wb = round256(wb + 2 * Bm * tmax);
  s->w_tb = wb;   wb = round256(wb + 2 * Bm * (w > fi ? w : fi));
  // largest split count <= 16 whose K range is a whole number of GEMM k steps
  s->splits = 1;
  for (int sp = 16; sp > 1; --sp)
    if (fo % (size_t(fks::kGemmKStep) * sp) == 0) {
      s->splits = sp;
      break;
    }
  s->w_sk = wb;   wb = round256(wb + 4 * size_t(s->splits) * Bm * w);
  s->w_w3t = wb;  wb = round256(wb + 2 * fo * w);  // W3 transposed ([width][n^3] bf16)
  s->ws_bytes = wb;
  *out = s;
  return ok();
}

fks_status fks_sur_sizes(fks_sur s, size_t* param_bytes, size_t* workspace_bytes, int64_t* n_params) {
  if (!s || !param_bytes || !workspace_bytes || !n_params) return fail(FKS_E_ARG, "null argument");
  *param_bytes = s->param_bytes;
  *workspace_bytes = s->ws_bytes;
  *n_params = int64_t(s->n_params);
  return ok();
}

fks_status fks_sur_bind(fks_sur s, void* d_params, size_t param_bytes, void* d_workspace, size_t workspace_bytes,
                        void* stream) {
  (void)stream;
  if (!s || !d_params || !d_workspace) return fail(FKS_E_ARG, "null argument");
  if (!aligned(d_params) || !aligned(d_workspace)) return fail(FKS_E_ARG, "buffers must be 256-byte aligned");
  if (param_bytes < s->param_bytes || workspace_bytes < s->ws_bytes) return fail(FKS_E_WORKSPACE, "buffers too small");
  s->d_params = d_params;
  s->d_ws = d_workspace;
  s->bound = true;
  return ok();
}

fks_status fks_sur_set_params(fks_sur s, const float* host, void* stream) {
  fks_status st = sur_ready(s);
  if (st != FKS_OK) return st;
  if (!host) return fail(FKS_E_ARG, "null params");
  hipStream_t hs = static_cast<hipStream_t>(stream);
  std::vector<uint16_t> h16(s->n_params);
  for (size_t i = 0; i < s->n_params; ++i) h16[i] = bf16_bits(host[i]);
  st = check_hip(hipMemcpyAsync(B(s->d_params, s->p_master), host, 4 * s->n_params, hipMemcpyHostToDevice, hs), "params");
  if (st == FKS_OK)
    st = check_hip(hipMemcpyAsync(B(s->d_params, s->p_w16), h16.data(), 2 * s->n_params, hipMemcpyHostToDevice, hs),
                   "params16");
  std::vector<float> zeros(s->n_params, 0.0f);
  if (st == FKS_OK)
    st = check_hip(hipMemcpyAsync(B(s->d_params, s->p_m), zeros.data(), 4 * s->n_params, hipMemcpyHostToDevice, hs), "m");
  if (st == FKS_OK)
    st = check_hip(hipMemcpyAsync(B(s->d_params, s->p_v), zeros.data(), 4 * s->n_params, hipMemcpyHostToDevice, hs), "v");
  if (st == FKS_OK) st = check_hip(hipStreamSynchronize(hs), "params sync");  // host vectors go out of scope
  s->adam_t = 0;
  return st == FKS_OK ? ok() : st;
}

fks_status fks_sur_get(fks_sur s, int32_t which, float* host, void* stream) {
  fks_status st = sur_ready(s);
  if (st != FKS_OK) return st;
  if (!host || which < 0 || which > 1) return fail(FKS_E_ARG, "bad arguments");
  const size_t off = which == 0 ? s->p_master : s->p_g;
  st = check_hip(hipMemcpyAsync(host, B(s->d_params, off), 4 * s->n_params, hipMemcpyDeviceToHost,
                                static_cast<hipStream_t>(stream)),
                 "copy out");
  if (st == FKS_OK) st = check_hip(hipStreamSynchronize(static_cast<hipStream_t>(stream)), "sync");
  return st == FKS_OK ? ok() : st;
}

fks_status fks_sur_features(fks_sur s, fks_plan p, const void* f, void* x, float* rho, double* mom, int64_t n_cells,
                            void* stream) {
  fks_status st = sur_ready(s);
  if (st != FKS_OK) return st;
  st = check_plan_ready(p);
  if (st != FKS_OK) return st;
  if (p->n != s->n) return fail(FKS_E_ARG, "plan and surrogate grids differ");
  if (n_cells < 0 || (n_cells > 0 && (!f || !x || !rho))) return fail(FKS_E_ARG, "bad buffers");
  if (s->center && n_cells > 0 && !mom) return fail(FKS_E_ARG, "a centred surrogate needs the moments buffer");
  if (n_cells == 0) return ok();
  if (n_cells > (int64_t(1) << 31) - 1) return fail(FKS_E_ARG, "too many cells");
  const double dv = 2.0 * p->d.L / p->n;
  const size_t cell_bytes = size_t(p->n) * p->n * p->n * p->esize;
  const int f32 = p->d.dtype == FKS_F32;
  // pruned transform of the kept modes (one pass over f, moments included) where compiled
  const hipError_t e = fks::launch_features(f32, p->n, s->modes, f, x, s->fin, rho, mom, s->center ? 1 : 0, p->d.L,
                                            n_cells, stream);
  if (e != hipErrorNotSupported) {
    st = check_hip(e, "features");
    return st == FKS_OK ? ok() : st;
  }
  // other grids: full transform, then the low modes
  if (!p->d_ws) return fail(FKS_E_STATE, "plan workspace not bound (fks_plan_bind with a workspace)");
  const double box3 = 8.0 * p->d.L * p->d.L * p->d.L;
  unsigned char* ws = static_cast<unsigned char*>(p->d_ws);
  for (int64_t c0 = 0; c0 < n_cells; c0 += p->max_cells) {
    const int64_t c = (n_cells - c0 < p->max_cells) ? (n_cells - c0) : p->max_cells;
    st = check_hip(fks::launch_forward(f32, p->n, static_cast<const unsigned char*>(f) + size_t(c0) * cell_bytes,
                                       ws + p->off_fhat, ws + p->off_scr, c, stream),
                   "feature transform");
    if (st != FKS_OK) return st;
    if (mom) {
      st = check_hip(fks::launch_moments(f32, p->n, static_cast<const unsigned char*>(f) + size_t(c0) * cell_bytes, c,
                                         mom + size_t(c0) * 5, p->d.L, dv, stream),
                     "moments");
      if (st != FKS_OK) return st;
    }
    st = check_hip(fks::launch_lowmodes(f32, ws + p->off_fhat, p->geo.table_rows, p->n / 2, p->geo.npair, p->K, p->Kh,
                                        s->modes / 2, box3, static_cast<unsigned char*>(x) + size_t(c0) * 2 * s->fin,
                                        s->fin, rho + c0, s->center ? mom + size_t(c0) * 5 : nullptr, p->d.L, c,
                                        stream),
                   "low modes");
    if (st != FKS_OK) return st;
  }
  return ok();
}

fks_status fks_sur_targets(fks_sur s, fks_plan p, const float* q, const float* rho, const double* mom, float* t,
                           int64_t n_cells, void* stream) {
  fks_status st = sur_ready(s);
  if (st != FKS_OK) return st;
  st = check_plan_ready(p);
  if (st != FKS_OK) return st;
  if (p->n != s->n) return fail(FKS_E_ARG, "plan and surrogate grids differ");
  if (n_cells < 0 || (n_cells > 0 && (!q || !rho || !t))) return fail(FKS_E_ARG, "bad buffers");
  if (s->center && n_cells > 0 && !mom) return fail(FKS_E_ARG, "a centred surrogate needs the moments");
  if (n_cells == 0) return ok();
  if (n_cells > (int64_t(1) << 31) - 1) return fail(FKS_E_ARG, "too many cells");
  if (s->center)
    st = check_hip(fks::launch_shift(s->n, q, s->fout, t, mom, +1, p->d.L, rho, s->scale, 2, nullptr, 0, n_cells, stream),
                   "centred targets");
  else
    st = check_hip(fks::launch_sur_target(q, rho, 1.0f / s->scale, t, s->fout, n_cells, stream), "targets");
  return st == FKS_OK ? ok() : st;
}

fks_status fks_sur_forward(fks_sur s, const void* x, float* y, int64_t batch, void* stream) {
  fks_status st = sur_ready(s);
  if (st != FKS_OK) return st;
  if (!x || !y || batch < 128 || batch % 128 || batch > s->max_batch)
    return fail(FKS_E_ARG, "batch must be a multiple of 128 up to max_batch");
  st = sur_forward(s, x, batch, stream, y);
  return st == FKS_OK ? ok() : st;
}

fks_status fks_sur_train_step(fks_sur s, const void* x, const float* t, int64_t batch, float lr, int32_t update,
                              double* d_loss, void* stream) {
  fks_status st = sur_ready(s);
  if (st != FKS_OK) return st;
  if (!x || !t || batch < 128 || batch % 128 || batch > s->max_batch)
    return fail(FKS_E_ARG, "batch must be a multiple of 128 up to max_batch");
  if (!(lr >= 0.0f) || !std::isfinite(lr)) return fail(FKS_E_ARG, "bad learning rate");
  st = sur_forward(s, x, batch, stream);
  if (st == FKS_OK) st = sur_backward(s, x, t, batch, d_loss, stream);
  if (st != FKS_OK || !update) return st == FKS_OK ? ok() : st;
  s->adam_t += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = float(1.0 - std::pow(0.9, double(s->adam_t))), c2 = float(1.0 - std::pow(0.999, double(s->adam_t)));
  float* P = reinterpret_cast<float*>(B(s->d_params, s->p_master));
  float* M = reinterpret_cast<float*>(B(s->d_params, s->p_m));
  float* V = reinterpret_cast<float*>(B(s->d_params, s->p_v));
  float* G = reinterpret_cast<float*>(B(s->d_params, s->p_g));
  unsigned char* W16 = B(s->d_params, s->p_w16);
  for (int l = 0; l < 3 && st == FKS_OK; ++l) {
    const size_t nw = s->off_b[l] - s->off_w[l];
    const size_t nb = (l < 2 ? s->off_w[l + 1] : s->n_params) - s->off_b[l];
    st = check_hip(fks::launch_adam(P + s->off_w[l], M + s->off_w[l], V + s->off_w[l], G + s->off_w[l],
                                    W16 + 2 * s->off_w[l], int64_t(nw), lr, b1, b2, eps, c1, c2, stream),
                   "adam W");
    if (st == FKS_OK)
      st = check_hip(fks::launch_adam(P + s->off_b[l], M + s->off_b[l], V + s->off_b[l], G + s->off_b[l], nullptr,
                                      int64_t(nb), lr, b1, b2, eps, c1, c2, stream),
                     "adam b");
  }
  return st == FKS_OK ? ok() : st;
}

// Surrogate inference with the spectral fallback, per chunk of max_batch cells.  ranked = 0:
// the cells whose relative moment residual exceeds `level` (a threshold) fall back;
// ranked = 1: the ceil(level * c) cells of each chunk of c cells with the largest absolute
// residual (relative residual times ||q_sur||_2) fall back.
static fks_status sur_infer_impl(fks_sur s, fks_plan p, const void* f, float* q, int64_t n_cells, int ranked,
                                 double level, int64_t* n_fallback, double* d_indicator, void* stream) {
  fks_status st = sur_ready(s);
  if (st != FKS_OK) return st;
  st = check_plan_ready(p);
  if (st != FKS_OK) return st;
  if (p->n != s->n || p->d.dtype != FKS_F32) return fail(FKS_E_ARG, "fallback plan must be FP32 on the same grid");
  if (n_cells < 0 || (n_cells > 0 && (!f || !q))) return fail(FKS_E_ARG, "bad buffers");
  if (n_cells > 0 && ranges_overlap(f, q, size_t(n_cells) * s->fout * 4)) return fail(FKS_E_ARG, "q must not overlap f");
  if (ranked && !(level >= 0.0 && level <= 1.0)) return fail(FKS_E_ARG, "fallback fraction must be in [0, 1]");
  if (n_fallback) *n_fallback = 0;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  const int n3 = s->fout;
  const size_t cell_bytes = size_t(n3) * 4;
  std::vector<double> h_r;
  for (int64_t c0 = 0; c0 < n_cells; c0 += s->max_batch) {
    const int64_t c = (n_cells - c0 < s->max_batch) ? (n_cells - c0) : s->max_batch;
    const int64_t rows = (c + 127) / 128 * 128;
    const unsigned char* fc = static_cast<const unsigned char*>(f) + size_t(c0) * cell_bytes;
    float* qc = q + size_t(c0) * n3;
    float* rho = reinterpret_cast<float*>(B(s->d_ws, s->w_rho));
    double* r = d_indicator ? d_indicator + c0 : reinterpret_cast<double*>(B(s->d_ws, s->w_r));
    double* mom = s->center ? reinterpret_cast<double*>(B(s->d_ws, s->w_mom)) : nullptr;
    st = fks_sur_features(s, p, fc, B(s->d_ws, s->w_x), rho, mom, c, stream);
    if (st == FKS_OK) st = sur_forward(s, B(s->d_ws, s->w_x), rows, stream);
    if (st == FKS_OK) {
      const float* y = reinterpret_cast<const float*>(B(s->d_ws, s->w_y));
      if (s->center)  // back from the mean-velocity frame: q(v) = scale rho^2 y(v - u)
        st = check_hip(fks::launch_shift(s->n, y, n3, qc, mom, -1, p->d.L, rho, s->scale, 1, r, ranked, c, stream),
                       "surrogate output");
      else
        st = check_hip(fks::launch_sur_output(y, n3, rho, s->scale, s->n, p->d.L, qc, r, ranked, c, stream),
                       "surrogate output");
    }
    if (st != FKS_OK) return st;
    double thr = level;
    if (ranked) {
      // the k-th largest absolute residual of the chunk on the host (the chunk is
      // synchronised once anyway, for the fallback count); the k cells above the next
      // smaller value fall back (ties at the boundary all fall back; NaN always does)
      const int64_t k = int64_t(std::ceil(level * double(c)));
      if (k <= 0) continue;
      h_r.resize(size_t(c));
      st = check_hip(hipMemcpyAsync(h_r.data(), r, size_t(c) * 8, hipMemcpyDeviceToHost, hs), "indicator copy");
      if (st == FKS_OK) st = check_hip(hipStreamSynchronize(hs), "indicator sync");
      if (st != FKS_OK) return st;
      for (double& v : h_r)
        if (std::isnan(v)) v = HUGE_VAL;
      std::nth_element(h_r.begin(), h_r.begin() + (k - 1), h_r.end(), std::greater<double>());
      thr = std::nextafter(h_r[size_t(k - 1)], -HUGE_VAL);
    } else if (!(level >= 0.0)) {
      continue;  // negative threshold: no fallback
    }
    int* list = reinterpret_cast<int*>(B(s->d_ws, s->w_list));
    int* cnt = reinterpret_cast<int*>(B(s->d_ws, s->w_cnt));
    st = check_hip(fks::launch_compact(r, int(c), thr, list, cnt, stream), "compact");
    int h_cnt = 0;
    if (st == FKS_OK) st = check_hip(hipMemcpyAsync(&h_cnt, cnt, 4, hipMemcpyDeviceToHost, hs), "count");
    if (st == FKS_OK) st = check_hip(hipStreamSynchronize(hs), "count sync");
    if (st != FKS_OK) return st;
    if (h_cnt > 0) {
      float* gf = reinterpret_cast<float*>(B(s->d_ws, s->w_gf));
      float* gq = reinterpret_cast<float*>(B(s->d_ws, s->w_gq));
      st = check_hip(fks::launch_gather_cells(0, reinterpret_cast<const float*>(fc), gf, list, h_cnt, n3, stream), "gather");
      if (st == FKS_OK) st = run_collide(p, gf, nullptr, gq, nullptr, 0.0, h_cnt, nullptr, stream);
      if (st == FKS_OK) st = check_hip(fks::launch_gather_cells(1, gq, qc, list, h_cnt, n3, stream), "scatter");
      if (st != FKS_OK) return st;
    }
    if (n_fallback) *n_fallback += h_cnt;
  }
  return ok();
}

fks_status fks_sur_infer(fks_sur s, fks_plan p, const void* f, float* q, int64_t n_cells, double threshold,
                         int64_t* n_fallback, double* d_indicator, void* stream) {
  return sur_infer_impl(s, p, f, q, n_cells, 0, threshold, n_fallback, d_indicator, stream);
}

fks_status fks_sur_infer_ranked(fks_sur s, fks_plan p, const void* f, float* q, int64_t n_cells,
                                double fallback_frac, int64_t* n_fallback, double* d_indicator, void* stream) {
  return sur_infer_impl(s, p, f, q, n_cells, 1, fallback_frac, n_fallback, d_indicator, stream);
}

void fks_sur_destroy(fks_sur s) { delete s; }

fks_status fks_graph_begin(void* stream) {
  return check_hip(hipStreamBeginCapture(static_cast<hipStream_t>(stream), hipStreamCaptureModeThreadLocal),
                   "begin capture") == FKS_OK
             ? ok()
             : FKS_E_DEVICE;
}

fks_status fks_graph_end(void* stream, fks_graph* out) {
  if (!out) return fail(FKS_E_ARG, "null out");
  *out = nullptr;
  hipGraph_t g = nullptr;
  fks_status s = check_hip(hipStreamEndCapture(static_cast<hipStream_t>(stream), &g), "end capture");
  if (s != FKS_OK) return s;
  hipGraphExec_t e = nullptr;
  s = check_hip(hipGraphInstantiate(&e, g, nullptr, nullptr, 0), "graph instantiate");
  if (s != FKS_OK) {
    (void)hipGraphDestroy(g);
    return s;
  }
  fks_graph_s* h = new (std::nothrow) fks_graph_s();
  if (!h) {
    (void)hipGraphExecDestroy(e);
    (void)hipGraphDestroy(g);
    return fail(FKS_E_ARG, "out of host memory");
  }
  h->graph = g;
  h->exec = e;
  *out = h;
  return ok();
}

fks_status fks_graph_launch(fks_graph g, void* stream) {
  if (!g) return fail(FKS_E_ARG, "null graph");
  return check_hip(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)), "graph launch") == FKS_OK ? ok()
                                                                                                  : FKS_E_DEVICE;
}

void fks_graph_destroy(fks_graph g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

fks_status fks_xport_create(int32_t n, double L, int32_t nx, int32_t ny, int32_t nz, double dx, fks_xport* out) {
  if (!out) return fail(FKS_E_ARG, "null out");
  *out = nullptr;
  if (n != 8 && n != 12 && n != 16 && n != 24 && n != 32)
    return fail(FKS_E_UNSUPPORTED, "transport velocity grids: n in {8, 12, 16, 24, 32}, got %d", n);
  if (nx < 1 || ny < 1 || nz < 1) return fail(FKS_E_ARG, "box sizes must be >= 1");
  if (int64_t(nx) * ny * nz > (int64_t(1) << 24)) return fail(FKS_E_ARG, "too many cells");
  // the per-cell kernels address a y-z plane of the box with 32-bit offsets
  if (int64_t(ny) * nz * int64_t(n) * n * n >= (int64_t(1) << 31))
    return fail(FKS_E_UNSUPPORTED, "a y-z plane of the box must hold fewer than 2^31 values (ny nz n^3)");
  if (!(L > 0.0) || !(dx > 0.0) || !std::isfinite(L) || !std::isfinite(dx))
    return fail(FKS_E_ARG, "L and dx must be positive");
  fks_xport_s* x = new (std::nothrow) fks_xport_s();
  if (!x) return fail(FKS_E_ARG, "out of host memory");
  x->n = n;
  x->L = L;
  x->nx = nx;
  x->ny = ny;
  x->nz = nz;
  x->dx = dx;
  *out = x;
  return ok();
}

fks_status fks_xport_sizes(fks_xport x, size_t* state_bytes) {
  if (!x || !state_bytes) return fail(FKS_E_ARG, "null argument");
  const size_t nv = size_t(x->n) * x->n * x->n;
  *state_bytes = round256(nv * 3 * 8) + round256(nv * 3 * 4) + round256(nv * 3 * 4) + round256(size_t(x->n) * 3 * 4);
  return ok();
}

static fks::XportState xport_state(fks_xport x) {
  const size_t nv = size_t(x->n) * x->n * x->n;
  unsigned char* b = static_cast<unsigned char*>(x->d_state);
  fks::XportState st;
  st.s = reinterpret_cast<double*>(b);
  st.o = reinterpret_cast<int32_t*>(b + round256(nv * 3 * 8));
  st.dl = reinterpret_cast<int32_t*>(b + round256(nv * 3 * 8) + round256(nv * 3 * 4));
  st.d1 = reinterpret_cast<int32_t*>(b + round256(nv * 3 * 8) + 2 * round256(nv * 3 * 4));
  return st;
}

fks_status fks_xport_bind(fks_xport x, void* d_state, size_t state_bytes, void* stream) {
  if (!x || !d_state) return fail(FKS_E_ARG, "null argument");
  if (!aligned(d_state)) return fail(FKS_E_ARG, "state must be 256-byte aligned");
  size_t need = 0;
  fks_xport_sizes(x, &need);
  if (state_bytes < need) return fail(FKS_E_WORKSPACE, "state buffer %zu < %zu bytes", state_bytes, need);
  x->d_state = d_state;
  x->bound = true;
  return check_hip(fks::launch_xport_reset(xport_state(x), x->n, stream), "transport reset") ==
                 FKS_OK
             ? ok()
             : FKS_E_DEVICE;
}

fks_status fks_transport_ex(fks_xport x, const void* f_in, void* f_out, int32_t dtype, double dt,
                            int32_t materialize, void* stream) {
  if (!x) return fail(FKS_E_ARG, "null transport");
  if (!x->bound) return fail(FKS_E_STATE, "transport state not bound");
  if (!std::isfinite(dt)) return fail(FKS_E_ARG, "dt must be finite");
  const int nv = x->n * x->n * x->n;
  if (materialize) {
    if (!f_in || !f_out) return fail(FKS_E_ARG, "null f_in or f_out");
    if (dtype != FKS_F32 && dtype != FKS_F64) return fail(FKS_E_ARG, "bad dtype");
    const size_t bytes = size_t(x->nx) * x->ny * x->nz * nv * (dtype == FKS_F32 ? 4 : 8);
    if (ranges_overlap(f_in, f_out, bytes)) return fail(FKS_E_ARG, "f_out must not overlap f_in");
  }
  const fks::XportState st = xport_state(x);
  fks_status s = check_hip(fks::launch_xport_advance(st, x->n, x->L, dt, x->dx, stream), "transport advance");
  if (s != FKS_OK || !materialize) return s == FKS_OK ? ok() : s;
  s = check_hip(fks::launch_roll(dtype == FKS_F32, f_in, f_out, st.d1, x->n, x->L, x->nx, x->ny, x->nz, stream),
                "transport roll");
  return s == FKS_OK ? ok() : s;
}

fks_status fks_transport(fks_xport x, const void* f_in, void* f_out, int32_t dtype, double dt, void* stream) {
  return fks_transport_ex(x, f_in, f_out, dtype, dt, 1, stream);
}

fks_status fks_step(fks_plan p, fks_xport x, void* f, void* f_tmp, double dt, int32_t n_steps, double* d_moments,
                    void* stream) {
  fks_status s = check_plan_ready(p);
  if (s != FKS_OK) return s;
  if (!x) return fail(FKS_E_ARG, "null transport");
  if (!x->bound) return fail(FKS_E_STATE, "transport state not bound");
  if (x->n != p->n || std::fabs(x->L - p->d.L) > 0.0) return fail(FKS_E_ARG, "plan and transport grids differ");
  if (!f || !f_tmp) return fail(FKS_E_ARG, "null f or f_tmp");
  if (n_steps < 0) return fail(FKS_E_ARG, "n_steps < 0");
  const int64_t cells = int64_t(x->nx) * x->ny * x->nz;
  const size_t bytes = size_t(cells) * p->n * p->n * p->n * p->esize;
  if (ranges_overlap(f, f_tmp, bytes)) return fail(FKS_E_ARG, "f_tmp must not overlap f");
  for (int st = 0; st < n_steps; ++st) {
    s = fks_transport(x, f, f_tmp, p->d.dtype, dt, stream);
    if (s != FKS_OK) return s;
    s = run_collide(p, f_tmp, f_tmp, nullptr, f, dt, cells, st == n_steps - 1 ? d_moments : nullptr, stream);
    if (s != FKS_OK) return s;
  }
  return ok();
}

fks_status fks_step_ex(fks_plan p, fks_xport x, void* f, void* f_tmp, double dt, int32_t n_steps,
                       const fks_step_opts* opts, void* stream) {
  fks_step_opts o{};
  if (opts) o = *opts;
  if (!p) return fail(FKS_E_ARG, "null plan");
  if (o.collision != FKS_COLL_BOLTZMANN && o.collision != FKS_COLL_BGK) return fail(FKS_E_ARG, "unknown collision");
  if (o.integrator != FKS_INT_EULER && o.integrator != FKS_INT_EXP) return fail(FKS_E_ARG, "unknown integrator");
  const bool bgk = o.collision == FKS_COLL_BGK;
  if (!bgk) {
    fks_status s = check_plan_ready(p);
    if (s != FKS_OK) return s;
  }
  if (!x) return fail(FKS_E_ARG, "null transport");
  if (!x->bound) return fail(FKS_E_STATE, "transport state not bound");
  if (x->n != p->n || std::fabs(x->L - p->d.L) > 0.0) return fail(FKS_E_ARG, "plan and transport grids differ");
  if (!f || !f_tmp) return fail(FKS_E_ARG, "null f or f_tmp");
  if (n_steps < 0) return fail(FKS_E_ARG, "n_steps < 0");
  if (!std::isfinite(dt)) return fail(FKS_E_ARG, "dt must be finite");
  if (bgk && (!(o.nu > 0.0) || !std::isfinite(o.nu))) return fail(FKS_E_ARG, "BGK needs nu > 0");
  if (bgk && !o.d_cons) return fail(FKS_E_ARG, "BGK needs the conservative variables d_cons");
  if (!bgk && o.integrator == FKS_INT_EXP && (!(o.mu > 0.0) || !std::isfinite(o.mu)))
    return fail(FKS_E_ARG, "the exponential Boltzmann step needs mu > 0");
  const int64_t cells = int64_t(x->nx) * x->ny * x->nz;
  const size_t bytes = size_t(cells) * p->n * p->n * p->n * p->esize;
  if (ranges_overlap(f, f_tmp, bytes)) return fail(FKS_E_ARG, "f_tmp must not overlap f");
  if (o.q_last && (ranges_overlap(o.q_last, f, bytes) || ranges_overlap(o.q_last, f_tmp, bytes)))
    return fail(FKS_E_ARG, "q_last must not overlap f or f_tmp");
  if (n_steps == 0) return ok();
  const int f32 = p->d.dtype == FKS_F32;
  const fks::XportState xs = xport_state(x);
  fks::StepCellArgs a{};
  a.n = p->n;
  a.L = p->d.L;
  a.nx = x->nx;
  a.ny = x->ny;
  a.nz = x->nz;
  a.cons = o.d_cons;
  a.prim = o.d_prim;
  a.nu = o.nu;
  a.nu_density = o.nu_density ? 1 : 0;
  a.dt = dt;
  fks_status s = FKS_OK;
  if (bgk) {
    // ping-pong between f and f_tmp; the fused kernel shifts, updates U and relaxes
    const int mode = o.integrator == FKS_INT_EXP ? 2 : 1;
    void* cur = f;
    void* nxt = f_tmp;
    for (int st = 0; st < n_steps && s == FKS_OK; ++st) {
      const bool last = st == n_steps - 1;
      s = check_hip(fks::launch_xport_advance(xs, x->n, x->L, dt, x->dx, stream), "transport advance");
      if (s != FKS_OK) break;
      a.q = last ? o.q_last : nullptr;
      a.moments = last ? o.d_moments : nullptr;
      s = check_hip(fks::launch_step_cell(f32, cur, nxt, xs.d1, mode, a, stream), "BGK step");
      std::swap(cur, nxt);
    }
    if (s == FKS_OK && cur != f)
      s = check_hip(fks::launch_copy(f32, cur, f, cells * int64_t(p->n) * p->n * p->n, stream), "copy back");
    return s == FKS_OK ? ok() : s;
  }
  const double dt_eff = o.integrator == FKS_INT_EXP ? -std::expm1(-o.mu * dt) / o.mu : dt;
  for (int st = 0; st < n_steps; ++st) {
    const bool last = st == n_steps - 1;
    s = check_hip(fks::launch_xport_advance(xs, x->n, x->L, dt, x->dx, stream), "transport advance");
    if (s != FKS_OK) return s;
    if (o.d_cons) {  // the shift with eq. DM_update from the masses before it
      a.q = nullptr;
      a.moments = nullptr;
      a.prim = last ? o.d_prim : nullptr;
      s = check_hip(fks::launch_step_cell(f32, f, f_tmp, xs.d1, 0, a, stream), "transport with DM update");
    } else {
      s = check_hip(fks::launch_roll(f32, f, f_tmp, xs.d1, x->n, x->L, x->nx, x->ny, x->nz, stream),
                    "transport roll");
    }
    if (s != FKS_OK) return s;
    double* mom = nullptr;
    if (last) mom = o.d_moments ? o.d_moments : (o.d_prim && !o.d_cons ? o.d_prim : nullptr);
    s = run_collide(p, f_tmp, f_tmp, last ? o.q_last : nullptr, f, dt_eff, cells, mom, stream);
    if (s != FKS_OK) return s;
  }
  if (o.d_prim && !o.d_cons)
    s = check_hip(fks::launch_to_primitive(o.d_moments ? o.d_moments : o.d_prim, o.d_prim, cells, stream),
                  "to primitive");
  return s == FKS_OK ? ok() : s;
}

void fks_xport_destroy(fks_xport x) { delete x; }

}  // extern "C"
