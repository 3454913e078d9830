// C ABI of the library: parameter validation, derived constants, launches.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <mutex>
#include <new>
#include <string>

#include "lbm_internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  g_err = std::string(where) + ": " + hipGetErrorString(e);
  return LBM_EHIP;
}

bool aligned(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// Per-step key of the stochastic rounding: the SplitMix64 output function of the
// step counter (a published generator), so consecutive steps draw unrelated bits.
uint32_t step_key(uint64_t seq) {
  uint64_t z = seq + 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return (uint32_t)(z ^ (z >> 31));
}

// Before every step launch: the step's rounding key, then the counter moves on.
void next_step(lbm_handle* h) { h->k.seq_hash = step_key(h->seq++); }

}  // namespace

// ------------------------------------------------------------ allocation-free adjoint step
// The two work fields of lbm_step_adjoint_full at the exact time level (the density, float[n], then
// the gradient cotangent, float[3 n], from the next 256-byte boundary) live in this static array, so
// that lbm_step_adjoint_full_noalloc allocates nothing.  Each device holds its own copy from module
// load to process exit; host code reaches it only through the address hipGetSymbolAddress returns
// for the current device (the array's name is a host-side stand-in).
static constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) float scratch[kScratchBytes / sizeof(float)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// floats of the array one call on an n-node grid uses
size_t noalloc_floats(int64_t n) { return (size_t)((n + 63) / 64 * 64) + 3 * (size_t)n; }

// The current device's copy of scratch, looked up on the first call on that device.
hipError_t scratch_here(float** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<float*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

const char* lbm_last_error(void) { return g_err.c_str(); }

int lbm_relaxation_rates(double nu, double xi, double cs2, double* omega_nu, double* omega_xi) {
  g_err.clear();
  if (omega_nu == nullptr || omega_xi == nullptr) return fail(LBM_EINVAL, "lbm_relaxation_rates: NULL output");
  if (!(nu > 0.0) || !(xi > 0.0) || !(cs2 > 0.0) || !std::isfinite(nu) || !std::isfinite(xi) || !std::isfinite(cs2))
    return fail(LBM_EINVAL, "lbm_relaxation_rates: nu, xi and cs2 must be finite and > 0");
  *omega_nu = 1.0 / (nu / cs2 + 0.5);
  *omega_xi = 1.0 / (1.5 * xi / cs2 + 0.5);
  return LBM_OK;
}

int lbm_create(const lbm_params* p, lbm_handle** out) {
  g_err.clear();
  if (p == nullptr || out == nullptr) return fail(LBM_EINVAL, "lbm_create: NULL argument");
  *out = nullptr;
  lbm_params q = *p;
  if (q.nx < 1 || q.ny < 1 || q.nz < 1) return fail(LBM_EINVAL, "lbm_create: grid sizes must be >= 1");
  const int32_t bcs[3] = {q.bc_x, q.bc_y, q.bc_z};
  const int32_t sizes[3] = {q.nx, q.ny, q.nz};
  for (int d = 0; d < 3; ++d) {
    if (bcs[d] != LBM_PERIODIC && bcs[d] != LBM_BOUNCEBACK) return fail(LBM_EINVAL, "lbm_create: unknown boundary type");
    if (bcs[d] == LBM_BOUNCEBACK && sizes[d] < 2)
      return fail(LBM_EINVAL, "lbm_create: a bounce-back axis needs at least 2 nodes");
  }
  int moving = 0;  // bit f: face f moves
  for (int f = 0; f < 6; ++f) {
    for (int c = 0; c < 3; ++c) {
      const double v = q.wall_velocity[f][c];
      if (!std::isfinite(v)) return fail(LBM_EINVAL, "lbm_create: non-finite wall velocity");
      if (v == 0.0) continue;
      if (bcs[f / 2] != LBM_BOUNCEBACK) return fail(LBM_EINVAL, "lbm_create: wall velocity on a periodic axis");
      if (c == f / 2) return fail(LBM_EINVAL, "lbm_create: wall velocity along the face normal");
      moving |= 1 << f;
    }
  }
  const int64_t n = (int64_t)q.nx * q.ny * q.nz;
  if (n > 0x7fffffffLL) return fail(LBM_EINVAL, "lbm_create: more than 2^31-1 nodes");
  if (!(q.r > 0.0) || !(q.s > 0.0)) return fail(LBM_EINVAL, "lbm_create: r and s must be > 0");
  if (!(q.cs2 > 0.0)) q.cs2 = std::fmin(q.r * q.r, q.s * q.s) / 3.0;
  if (!(q.cs2 < 1.0 && q.cs2 < q.r * q.r && q.cs2 < q.s * q.s))
    return fail(LBM_EINVAL, "lbm_create: cs2 must be < min(1, r^2, s^2) (positive rest weights)");
  if (!(q.omega_nu > 0.0 && q.omega_nu < 2.0) || !(q.omega_xi > 0.0 && q.omega_xi < 2.0))
    return fail(LBM_EINVAL, "lbm_create: omega_nu and omega_xi must lie in (0, 2)");
  if (!(q.omega_hi > 0.0 && q.omega_hi < 2.0))
    return fail(LBM_EINVAL, "lbm_create: omega_hi must lie in (0, 2)");
  if (q.storage < LBM_F32 || q.storage > LBM_BF16_SR) return fail(LBM_EINVAL, "lbm_create: unknown storage");
  if (q.corr < LBM_CORR_OFF || q.corr > LBM_CORR_FULL) return fail(LBM_EINVAL, "lbm_create: unknown correction");
  if (q.moments != LBM_CENTRAL && q.moments != LBM_RAW) return fail(LBM_EINVAL, "lbm_create: unknown moment basis");
  if (q.layout != LBM_LAYOUT_AB && q.layout != LBM_LAYOUT_AA) return fail(LBM_EINVAL, "lbm_create: unknown layout");
  if (q.layout == LBM_LAYOUT_AA && q.corr == LBM_CORR_FULL)
    return fail(LBM_EINVAL, "lbm_create: the AA layout does not run the full corrections");
  if (!(q.rho0 > 0.0)) return fail(LBM_EINVAL, "lbm_create: rho0 must be > 0");
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(q.force[d])) return fail(LBM_EINVAL, "lbm_create: non-finite force");

  lbm_handle* h = new (std::nothrow) lbm_handle();
  if (h == nullptr) return fail(LBM_EINVAL, "lbm_create: out of host memory");
  h->p = q;
  h->n = n;
  // blocked layout: every x-row padded to whole blocks of kB nodes
  const int64_t nxp = ((int64_t)q.nx + clbm::kB - 1) / clbm::kB * clbm::kB;
  h->stride = nxp * q.ny * q.nz;
  h->elem = q.storage == LBM_F32 ? 4 : 2;
  h->bytes = (size_t)27 * (size_t)h->stride * h->elem;
  // the AA kernels with walls address the state through 32-bit offsets
  if (q.layout == LBM_LAYOUT_AA && (q.bc_x == LBM_BOUNCEBACK || q.bc_y == LBM_BOUNCEBACK || q.bc_z == LBM_BOUNCEBACK) &&
      h->bytes >= (1ull << 32)) {
    delete h;
    return fail(LBM_EINVAL, "lbm_create: the AA layout with walls needs a state below 4 GiB");
  }
  // threads per block along x: of the candidates in order of preference, the
  // first that leaves the fewest idle lanes in the last block of a row (e.g. 192
  // for nx = 384).  The FP32 step without full corrections prefers 128 (measured
  // +1.5% at 512x512x256); the other kernels 256 (128 measured 1-2% slower).
  auto pick_block = [&](std::initializer_list<int> order) {
    int best = 256, best_waste = 1 << 30;
    for (int b : order) {
      const int waste = (q.nx + b - 1) / b * b - q.nx;
      if (waste < best_waste) { best_waste = waste; best = b; }
    }
    return best;
  };
  h->block = pick_block({256, 192, 128, 64});
  h->block_step = q.storage == LBM_F32 ? pick_block({128, 256, 192, 64}) : h->block;
  h->pairs = 1;
  if (const char* env = std::getenv("LBM_PAIRS")) h->pairs = std::atoi(env) != 0;  // 0: one node per thread
  h->seq = 0;
  h->force_kind = 0;
  if (const char* env = std::getenv("LBM_GATHER_KIND")) {  // testing: 1 or 2, taken where valid
    const int kind = std::atoi(env);
    if (kind == 1 || kind == 2) h->force_kind = kind;
  }
  // Occupancy caps through LDS the kernels do not use: a launch reserves
  // 160 KiB / (blocks per CU) so that at most `waves` waves per SIMD fit.  The
  // FP32 one-node steps fit 5 waves per SIMD in registers but run fastest at 3
  // (512x512x256: 2.481 ms at 3, 2.509 at 4, 2.531 at 5, 2.496 at 3.5); the
  // 16-bit ones are fastest unlimited.  LBM_STEP_LDS / LBM_PAIR_LDS override the
  // bytes per block (0 = no cap).
  auto lds_cap = [](int block, int waves) {
    const int blocks_per_cu = 4 * waves / (block / 64);
    return blocks_per_cu < 1 ? 0 : (163840 / blocks_per_cu) & ~511;
  };
  if (const char* env = std::getenv("LBM_BLOCK")) {
    const int b = std::atoi(env);
    if (b == 64 || b == 128 || b == 192 || b == 256) h->block = h->block_step = b;
  }
  h->step_lds = q.storage == LBM_F32 ? lds_cap(h->block_step, 3) : 0;
  if (const char* env = std::getenv("LBM_STEP_LDS")) {
    const int b = std::atoi(env);
    if (b >= 0 && b <= 65536) h->step_lds = b;
  }
  h->pair_lds = 0;
  if (const char* env = std::getenv("LBM_PAIR_LDS")) {
    const int b = std::atoi(env);
    if (b >= 0 && b <= 65536) h->pair_lds = b;
  }

  const double c[3] = {1.0, q.r, q.s};
  clbm::Consts& k = h->k;
  clbm::ConstsD& kd = h->kd;
  k.nx = q.nx; k.ny = q.ny; k.nz = q.nz;
  k.bb_x = q.bc_x == LBM_BOUNCEBACK;
  k.bb_y = q.bc_y == LBM_BOUNCEBACK;
  k.bb_z = q.bc_z == LBM_BOUNCEBACK;
  k.moving = moving;
  k.aa = q.layout == LBM_LAYOUT_AA ? 1 : 0;
  k.hi = q.omega_hi != 1.0 ? 1 : 0;
  k.ytile = 1;
  for (int t : {32, 16, 8, 4, 2})
    if (q.ny % t == 0) { k.ytile = t; break; }
  if (const char* env = std::getenv("LBM_FULL_YTILE")) {  // tuning: any divisor of ny (ny = plain row order)
    const int t = std::atoi(env);
    if (t >= 1 && q.ny % t == 0) k.ytile = t;
  }

  for (int f = 0; f < 6; ++f)
    for (int c = 0; c < 3; ++c) k.wall_u[f][c] = (float)q.wall_velocity[f][c];
  k.row_slots = 27 * nxp;
  k.n = n;
  k.rho0 = (float)q.rho0; k.cs2 = (float)q.cs2; k.r = (float)q.r; k.s = (float)q.s;
  k.omega_nu = (float)q.omega_nu; k.omega_xi = (float)q.omega_xi; k.omega_hi = (float)q.omega_hi;
  k.fx = (float)q.force[0]; k.fy = (float)q.force[1]; k.fz = (float)q.force[2];
  kd.rho0 = q.rho0; kd.cs2 = q.cs2;
  double W[3][3];
  for (int d = 0; d < 3; ++d) {
    const double c2 = c[d] * c[d];
    k.c2[d] = (float)c2;
    k.ic[d] = (float)(1.0 / c[d]);
    k.ic2[d] = (float)(1.0 / c2);
    kd.ic[d] = 1.0 / c[d];
    kd.ic2[d] = 1.0 / c2;
    kd.w0c[d] = 1.0 - q.cs2 / c2;
    kd.w0s[d] = q.cs2 / (2.0 * c2);
    k.w0c[d] = (float)kd.w0c[d];
    k.w0s[d] = (float)kd.w0s[d];
    W[d][0] = kd.w0s[d]; W[d][1] = kd.w0c[d]; W[d][2] = kd.w0s[d];
  }
  for (int a = 0; a < 27; ++a) {
    const double w = W[0][clbm::kEx[a] + 1] * W[1][clbm::kEy[a] + 1] * W[2][clbm::kEz[a] + 1];
    kd.w[a] = w;
    // power-of-two scale near 1/w for FP16 storage (exact, so it adds no rounding); FP32 and
    // BF16 share the FP32 exponent range and store unscaled deviations
    const double sig = q.storage == LBM_F16 ? std::ldexp(1.0, (int)std::lround(-std::log2(w))) : 1.0;
    k.sigma[clbm::wclass(a)] = (float)sig;          // equal within a weight class
    k.inv_sigma[clbm::wclass(a)] = (float)(1.0 / sig);
  }
  *out = h;
  return LBM_OK;
}

void lbm_destroy(lbm_handle* h) { delete h; }

size_t lbm_state_bytes(const lbm_handle* h) { return h ? h->bytes : 0; }
int64_t lbm_state_stride(const lbm_handle* h) { return h ? h->stride : 0; }
int64_t lbm_num_nodes(const lbm_handle* h) { return h ? h->n : 0; }

#define CHECK_HANDLE(h, name) \
  if ((h) == nullptr) return fail(LBM_ESTATE, name ": NULL handle")
#define CHECK_PTR(ptr, name, what) \
  if ((ptr) != nullptr && !aligned(ptr)) return fail(LBM_EINVAL, name ": " what " is not 16-byte aligned")
#define CHECK_REQ(ptr, name, what) \
  if ((ptr) == nullptr) return fail(LBM_EINVAL, name ": " what " is NULL"); \
  CHECK_PTR(ptr, name, what)

int lbm_set_step_counter(lbm_handle* h, uint64_t counter) {
  CHECK_HANDLE(h, "lbm_set_step_counter");
  h->seq = counter;
  return LBM_OK;
}

uint64_t lbm_step_counter(const lbm_handle* h) { return h ? h->seq : 0; }

int lbm_init(lbm_handle* h, void* state, const double* rho, const double* u, const double* perturb,
             void* hip_stream) {
  CHECK_HANDLE(h, "lbm_init");
  CHECK_REQ(state, "lbm_init", "state");
  CHECK_PTR(rho, "lbm_init", "rho");
  CHECK_PTR(u, "lbm_init", "u");
  CHECK_PTR(perturb, "lbm_init", "perturb");
  hipError_t e = clbm::launch_init(*h, state, rho, u, perturb, (hipStream_t)hip_stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_init");
}

int lbm_import(lbm_handle* h, void* state, const double* f, void* hip_stream) {
  CHECK_HANDLE(h, "lbm_import");
  CHECK_REQ(state, "lbm_import", "state");
  CHECK_REQ(f, "lbm_import", "f");
  hipError_t e = clbm::launch_import(*h, state, f, (hipStream_t)hip_stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_import");
}

int lbm_export(lbm_handle* h, const void* state, double* f, void* hip_stream) {
  CHECK_HANDLE(h, "lbm_export");
  CHECK_REQ(state, "lbm_export", "state");
  CHECK_REQ(f, "lbm_export", "f");
  hipError_t e = clbm::launch_export(*h, state, f, (hipStream_t)hip_stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_export");
}

int lbm_export_nodes(lbm_handle* h, const void* state, const int64_t* nodes, int64_t count, double* f,
                     void* hip_stream) {
  CHECK_HANDLE(h, "lbm_export_nodes");
  if (count < 0) return fail(LBM_EINVAL, "lbm_export_nodes: count < 0");
  if (count == 0) return LBM_OK;
  CHECK_REQ(state, "lbm_export_nodes", "state");
  CHECK_REQ(nodes, "lbm_export_nodes", "nodes");
  CHECK_REQ(f, "lbm_export_nodes", "f");
  hipError_t e = clbm::launch_export_nodes(*h, state, nodes, count, f, (hipStream_t)hip_stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_export_nodes");
}

// AA layout: one buffer, steps in pairs (local, shifted).
static int step_aa(lbm_handle* h, const char* name, int32_t nsteps, void* state, void* state_b,
                   const float* force, const double* forces, hipStream_t st) {
  if (state_b != nullptr && state_b != state)
    return fail(LBM_EINVAL, std::string(name) + ": the AA layout updates state_a in place (state_b must be NULL)");
  if (nsteps % 2 != 0) return fail(LBM_EINVAL, std::string(name) + ": the AA layout advances an even number of steps");
  for (int32_t t = 0; t < nsteps; ++t) {
    next_step(h);
    hipError_t e = forces ? clbm::launch_step_aa_uniform(*h, state, t & 1, (float)forces[3 * t],
                                                         (float)forces[3 * t + 1], (float)forces[3 * t + 2], st)
                          : clbm::launch_step_aa(*h, state, t & 1, force, st);
    if (e != hipSuccess) return hip_fail(e, name);
  }
  return LBM_OK;
}

int lbm_step(lbm_handle* h, int32_t nsteps, void* state_a, void* state_b, const float* force,
             void* hip_stream) {
  CHECK_HANDLE(h, "lbm_step");
  if (nsteps < 0) return fail(LBM_EINVAL, "lbm_step: nsteps < 0");
  CHECK_REQ(state_a, "lbm_step", "state_a");
  CHECK_PTR(force, "lbm_step", "force");
  if (h->k.aa) return step_aa(h, "lbm_step", nsteps, state_a, state_b, force, nullptr, (hipStream_t)hip_stream);
  CHECK_REQ(state_b, "lbm_step", "state_b");
  if (state_a == state_b) return fail(LBM_EINVAL, "lbm_step: state_a and state_b must differ");
  if (h->p.corr == LBM_CORR_FULL)
    return fail(LBM_EINVAL, "lbm_step: the full corrections need a density field (use lbm_step_full)");
  void* bufs[2] = {state_a, state_b};
  for (int32_t t = 0; t < nsteps; ++t) {
    next_step(h);
    hipError_t e = clbm::launch_step(*h, bufs[t & 1], bufs[(t + 1) & 1], force, nullptr, nullptr,
                                     (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "lbm_step");
  }
  return LBM_OK;
}

int lbm_set_force(lbm_handle* h, const double force[3]) {
  CHECK_HANDLE(h, "lbm_set_force");
  if (force == nullptr) return fail(LBM_EINVAL, "lbm_set_force: NULL force");
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(force[d])) return fail(LBM_EINVAL, "lbm_set_force: non-finite force");
  for (int d = 0; d < 3; ++d) h->p.force[d] = force[d];
  h->k.fx = (float)force[0];
  h->k.fy = (float)force[1];
  h->k.fz = (float)force[2];
  return LBM_OK;
}

int lbm_step_forcing(lbm_handle* h, int32_t nsteps, void* state_a, void* state_b, const double* forces,
                     void* hip_stream) {
  CHECK_HANDLE(h, "lbm_step_forcing");
  if (nsteps < 0) return fail(LBM_EINVAL, "lbm_step_forcing: nsteps < 0");
  CHECK_REQ(state_a, "lbm_step_forcing", "state_a");
  if (h->p.corr == LBM_CORR_FULL)
    return fail(LBM_EINVAL, "lbm_step_forcing: the full corrections need a density field (use lbm_step_full)");
  if (nsteps > 0 && forces == nullptr) return fail(LBM_EINVAL, "lbm_step_forcing: NULL forces");
  for (int64_t i = 0; i < 3 * (int64_t)nsteps; ++i)
    if (!std::isfinite(forces[i])) return fail(LBM_EINVAL, "lbm_step_forcing: non-finite force");
  if (h->k.aa)
    return step_aa(h, "lbm_step_forcing", nsteps, state_a, state_b, nullptr, forces, (hipStream_t)hip_stream);
  CHECK_REQ(state_b, "lbm_step_forcing", "state_b");
  if (state_a == state_b) return fail(LBM_EINVAL, "lbm_step_forcing: state_a and state_b must differ");
  void* bufs[2] = {state_a, state_b};
  for (int32_t t = 0; t < nsteps; ++t) {
    next_step(h);
    hipError_t e = clbm::launch_step_uniform(*h, bufs[t & 1], bufs[(t + 1) & 1], (float)forces[3 * t],
                                             (float)forces[3 * t + 1], (float)forces[3 * t + 2],
                                             (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "lbm_step_forcing");
  }
  return LBM_OK;
}

int lbm_density(lbm_handle* h, const void* state, float* drho, void* hip_stream) {
  CHECK_HANDLE(h, "lbm_density");
  CHECK_REQ(state, "lbm_density", "state");
  CHECK_REQ(drho, "lbm_density", "drho");
  hipError_t e = clbm::launch_density(*h, state, drho, (hipStream_t)hip_stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_density");
}

int lbm_step_full(lbm_handle* h, int32_t nsteps, void* state_a, void* state_b, const float* force,
                  float* drho_a, float* drho_b, int32_t mode, void* hip_stream) {
  CHECK_HANDLE(h, "lbm_step_full");
  if (h->p.corr != LBM_CORR_FULL) return fail(LBM_EINVAL, "lbm_step_full: the handle's corr is not LBM_CORR_FULL");
  if (nsteps < 0) return fail(LBM_EINVAL, "lbm_step_full: nsteps < 0");
  if (mode != LBM_GRAD_EXACT && mode != LBM_GRAD_LAGGED) return fail(LBM_EINVAL, "lbm_step_full: unknown mode");
  CHECK_REQ(state_a, "lbm_step_full", "state_a");
  CHECK_REQ(state_b, "lbm_step_full", "state_b");
  CHECK_PTR(force, "lbm_step_full", "force");
  CHECK_REQ(drho_a, "lbm_step_full", "drho_a");
  if (state_a == state_b) return fail(LBM_EINVAL, "lbm_step_full: state_a and state_b must differ");
  if (mode == LBM_GRAD_LAGGED) {
    CHECK_REQ(drho_b, "lbm_step_full", "drho_b");
    if (drho_a == drho_b) return fail(LBM_EINVAL, "lbm_step_full: drho_a and drho_b must differ");
  } else {
    CHECK_PTR(drho_b, "lbm_step_full", "drho_b");
  }
  const hipStream_t st = (hipStream_t)hip_stream;
  void* bufs[2] = {state_a, state_b};
  float* rho[2] = {drho_a, drho_b};
  for (int32_t t = 0; t < nsteps; ++t) {
    void* src = bufs[t & 1];
    void* dst = bufs[(t + 1) & 1];
    next_step(h);
    hipError_t e;
    if (mode == LBM_GRAD_EXACT) {
      e = clbm::launch_density(*h, src, drho_a, st);
      if (e == hipSuccess) e = clbm::launch_step(*h, src, dst, force, drho_a, nullptr, st);
    } else {
      e = clbm::launch_step(*h, src, dst, force, rho[t & 1], rho[(t + 1) & 1], st);
    }
    if (e != hipSuccess) return hip_fail(e, "lbm_step_full");
  }
  return LBM_OK;
}

int lbm_stream(lbm_handle* h, int32_t nsteps, void* state_a, void* state_b, void* hip_stream) {
  CHECK_HANDLE(h, "lbm_stream");
  if (nsteps < 0) return fail(LBM_EINVAL, "lbm_stream: nsteps < 0");
  if (h->k.aa) return fail(LBM_EINVAL, "lbm_stream: the AB layout only");
  if (h->k.moving) return fail(LBM_EINVAL, "lbm_stream: stationary walls only");
  CHECK_REQ(state_a, "lbm_stream", "state_a");
  CHECK_REQ(state_b, "lbm_stream", "state_b");
  if (state_a == state_b) return fail(LBM_EINVAL, "lbm_stream: state_a and state_b must differ");
  void* bufs[2] = {state_a, state_b};
  for (int32_t t = 0; t < nsteps; ++t) {
    hipError_t e = clbm::launch_stream(*h, bufs[t & 1], bufs[(t + 1) & 1], (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "lbm_stream");
  }
  return LBM_OK;
}

int lbm_adjoint_stream(lbm_handle* h, const void* state_t, const float* adj_in, float* adj_out, const float* force,
                       float* grad_force, void* hip_stream) {
  CHECK_HANDLE(h, "lbm_adjoint_stream");
  if (h->k.aa) return fail(LBM_EINVAL, "lbm_adjoint_stream: the AB layout only");
  CHECK_REQ(state_t, "lbm_adjoint_stream", "state_t");
  CHECK_REQ(adj_in, "lbm_adjoint_stream", "adj_in");
  CHECK_REQ(adj_out, "lbm_adjoint_stream", "adj_out");
  CHECK_PTR(force, "lbm_adjoint_stream", "force");
  CHECK_PTR(grad_force, "lbm_adjoint_stream", "grad_force");
  if ((const void*)adj_in == (const void*)adj_out) return fail(LBM_EINVAL, "lbm_adjoint_stream: adj_in == adj_out");
  const hipStream_t st = (hipStream_t)hip_stream;
  hipError_t e;
  switch (h->p.storage) {
    case LBM_F32: e = clbm::AdjointKernels<0>::stream(*h, state_t, adj_in, adj_out, force, grad_force, st); break;
    case LBM_F16: e = clbm::AdjointKernels<1>::stream(*h, state_t, adj_in, adj_out, force, grad_force, st); break;
    default: e = clbm::AdjointKernels<2>::stream(*h, state_t, adj_in, adj_out, force, grad_force, st); break;
  }
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_adjoint_stream");
}

int lbm_copy(void* dst, const void* src, size_t bytes, void* hip_stream) {
  g_err.clear();
  if (bytes == 0) return LBM_OK;
  CHECK_REQ(dst, "lbm_copy", "dst");
  CHECK_REQ(src, "lbm_copy", "src");
  if (bytes % 16 != 0) return fail(LBM_EINVAL, "lbm_copy: bytes must be a multiple of 16");
  const uintptr_t a = (uintptr_t)dst, b = (uintptr_t)src;
  if (a < b + bytes && b < a + bytes) return fail(LBM_EINVAL, "lbm_copy: src and dst overlap");
  hipError_t e = clbm::launch_copy(dst, src, bytes, (hipStream_t)hip_stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_copy");
}

int lbm_moments(lbm_handle* h, const void* state, const float* force, float* rho, float* u,
                double* sums, void* hip_stream) {
  CHECK_HANDLE(h, "lbm_moments");
  CHECK_REQ(state, "lbm_moments", "state");
  CHECK_PTR(force, "lbm_moments", "force");
  CHECK_PTR(rho, "lbm_moments", "rho");
  CHECK_PTR(u, "lbm_moments", "u");
  CHECK_PTR(sums, "lbm_moments", "sums");
  hipError_t e = clbm::launch_moments(*h, state, force, rho, u, sums, (hipStream_t)hip_stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_moments");
}

int lbm_check_sums(const double* sums_device, double* out_host, void* hip_stream) {
  if (sums_device == nullptr) return fail(LBM_EINVAL, "lbm_check_sums: NULL sums");
  double tmp[5];
  hipError_t e = hipMemcpyAsync(tmp, sums_device, sizeof(tmp), hipMemcpyDeviceToHost, (hipStream_t)hip_stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "lbm_check_sums");
  if (out_host) std::memcpy(out_host, tmp, sizeof(tmp));
  for (double v : tmp)
    if (!std::isfinite(v)) return fail(LBM_ENONFINITE, "lbm_check_sums: non-finite total");
  return LBM_OK;
}

int lbm_step_adjoint(lbm_handle* h, const void* state_t, const float* adj_in, float* adj_out,
                     const float* force, float* grad_force, double* grad_force_uniform, void* hip_stream) {
  CHECK_HANDLE(h, "lbm_step_adjoint");
  if (h->k.aa) return fail(LBM_EINVAL, "lbm_step_adjoint: the adjoint runs on the AB layout only");
  CHECK_REQ(state_t, "lbm_step_adjoint", "state_t");
  CHECK_REQ(adj_in, "lbm_step_adjoint", "adj_in");
  CHECK_REQ(adj_out, "lbm_step_adjoint", "adj_out");
  CHECK_PTR(force, "lbm_step_adjoint", "force");
  CHECK_PTR(grad_force, "lbm_step_adjoint", "grad_force");
  CHECK_PTR(grad_force_uniform, "lbm_step_adjoint", "grad_force_uniform");
  if ((const void*)adj_in == (const void*)adj_out) return fail(LBM_EINVAL, "lbm_step_adjoint: adj_in == adj_out");
  if (h->p.corr == LBM_CORR_FULL)
    return fail(LBM_EINVAL, "lbm_step_adjoint: the full corrections need lbm_step_adjoint_full");
  hipError_t e = clbm::launch_step_adjoint(*h, state_t, adj_in, adj_out, force, grad_force,
                                           grad_force_uniform, nullptr, nullptr, false, false, nullptr,
                                           (hipStream_t)hip_stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_step_adjoint");
}

int lbm_step_adjoint_full(lbm_handle* h, int32_t mode, const void* state_t, const float* adj_in, float* adj_out,
                          const float* force, float* grad_force, double* grad_force_uniform, float* drho,
                          float* grad_work, const float* grad_pending, void* hip_stream) {
  CHECK_HANDLE(h, "lbm_step_adjoint_full");
  if (h->k.aa) return fail(LBM_EINVAL, "lbm_step_adjoint_full: the adjoint runs on the AB layout only");
  if (h->p.corr != LBM_CORR_FULL)
    return fail(LBM_EINVAL, "lbm_step_adjoint_full: the handle's corrections are not LBM_CORR_FULL");
  if (mode != LBM_GRAD_EXACT && mode != LBM_GRAD_LAGGED && mode != LBM_GRAD_EXACT_DRHO)
    return fail(LBM_EINVAL, "lbm_step_adjoint_full: mode must be LBM_GRAD_EXACT, LBM_GRAD_EXACT_DRHO or LBM_GRAD_LAGGED");
  CHECK_REQ(state_t, "lbm_step_adjoint_full", "state_t");
  CHECK_REQ(adj_in, "lbm_step_adjoint_full", "adj_in");
  CHECK_REQ(adj_out, "lbm_step_adjoint_full", "adj_out");
  CHECK_REQ(drho, "lbm_step_adjoint_full", "drho");
  CHECK_REQ(grad_work, "lbm_step_adjoint_full", "grad_work");
  CHECK_PTR(grad_pending, "lbm_step_adjoint_full", "grad_pending");
  CHECK_PTR(force, "lbm_step_adjoint_full", "force");
  CHECK_PTR(grad_force, "lbm_step_adjoint_full", "grad_force");
  CHECK_PTR(grad_force_uniform, "lbm_step_adjoint_full", "grad_force_uniform");
  if ((const void*)adj_in == (const void*)adj_out)
    return fail(LBM_EINVAL, "lbm_step_adjoint_full: adj_in == adj_out");
  if ((const void*)drho == (const void*)grad_work)
    return fail(LBM_EINVAL, "lbm_step_adjoint_full: drho == grad_work");
  if (grad_pending != nullptr && (mode != LBM_GRAD_LAGGED || (const void*)grad_pending == (const void*)grad_work))
    return fail(LBM_EINVAL, "lbm_step_adjoint_full: grad_pending is for LBM_GRAD_LAGGED and must differ from grad_work");
  hipError_t e = clbm::launch_step_adjoint(*h, state_t, adj_in, adj_out, force, grad_force, grad_force_uniform,
                                           drho, grad_work, mode != LBM_GRAD_LAGGED, mode == LBM_GRAD_EXACT_DRHO,
                                           grad_pending,
                                           (hipStream_t)hip_stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_step_adjoint_full");
}

int lbm_density_adjoint(lbm_handle* h, const float* grad, float* adj, void* hip_stream) {
  CHECK_HANDLE(h, "lbm_density_adjoint");
  if (h->k.aa) return fail(LBM_EINVAL, "lbm_density_adjoint: the adjoint runs on the AB layout only");
  CHECK_REQ(grad, "lbm_density_adjoint", "grad");
  CHECK_REQ(adj, "lbm_density_adjoint", "adj");
  hipError_t e = clbm::launch_density_adjoint(*h, grad, adj, (hipStream_t)hip_stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_density_adjoint");
}

// The allocation-free variant of lbm_step_adjoint_full (exact time level): its work fields come
// from the static array above.
int lbm_step_adjoint_full_noalloc(lbm_handle* h, const void* state_t, const float* adj_in, float* adj_out,
                                  const float* force, float* grad_force, double* grad_force_uniform,
                                  void* hip_stream) {
  const char* name = "lbm_step_adjoint_full_noalloc";
  CHECK_HANDLE(h, "lbm_step_adjoint_full_noalloc");
  if (h->k.aa) return fail(LBM_EINVAL, std::string(name) + ": the adjoint runs on the AB layout only");
  if (h->p.corr != LBM_CORR_FULL)
    return fail(LBM_EINVAL, std::string(name) + ": the handle's corrections are not LBM_CORR_FULL");
  CHECK_REQ(state_t, "lbm_step_adjoint_full_noalloc", "state_t");
  CHECK_REQ(adj_in, "lbm_step_adjoint_full_noalloc", "adj_in");
  CHECK_REQ(adj_out, "lbm_step_adjoint_full_noalloc", "adj_out");
  CHECK_PTR(force, "lbm_step_adjoint_full_noalloc", "force");
  CHECK_PTR(grad_force, "lbm_step_adjoint_full_noalloc", "grad_force");
  CHECK_PTR(grad_force_uniform, "lbm_step_adjoint_full_noalloc", "grad_force_uniform");
  if ((const void*)adj_in == (const void*)adj_out) return fail(LBM_EINVAL, std::string(name) + ": adj_in == adj_out");
  const size_t need = noalloc_floats(h->n) * sizeof(float);
  if (need > kScratchBytes)
    return fail(LBM_EINVAL, std::string(name) + ": the grid's " + std::to_string(h->n) + " nodes need " +
                                std::to_string(need) + " bytes of work space, above the static array's " +
                                std::to_string(kScratchBytes) + " (at most " +
                                std::to_string(kScratchBytes / sizeof(float) / 4 - 16) +
                                " nodes); use lbm_step_adjoint_full with work fields instead");
  float* base = nullptr;
  hipError_t e = scratch_here(&base);
  if (e != hipSuccess) return hip_fail(e, name);
  float* drho = base;                                         // float[n], written by the density pass
  float* grad = base + (size_t)((h->n + 63) / 64 * 64);       // float[3 n], written by the adjoint kernel
  e = clbm::launch_step_adjoint(*h, state_t, adj_in, adj_out, force, grad_force, grad_force_uniform, drho, grad,
                                true, false, nullptr, (hipStream_t)hip_stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, name);
}

int lbm_moments_adjoint(lbm_handle* h, const void* state, const float* force, const float* g_rho,
                        const float* g_u, float* adj, float* grad_force, void* hip_stream) {
  CHECK_HANDLE(h, "lbm_moments_adjoint");
  if (h->k.aa) return fail(LBM_EINVAL, "lbm_moments_adjoint: the adjoint runs on the AB layout only");
  CHECK_REQ(state, "lbm_moments_adjoint", "state");
  CHECK_REQ(adj, "lbm_moments_adjoint", "adj");
  CHECK_PTR(force, "lbm_moments_adjoint", "force");
  CHECK_PTR(g_rho, "lbm_moments_adjoint", "g_rho");
  CHECK_PTR(g_u, "lbm_moments_adjoint", "g_u");
  CHECK_PTR(grad_force, "lbm_moments_adjoint", "grad_force");
  hipError_t e = clbm::launch_moments_adjoint(*h, state, force, g_rho, g_u, adj, grad_force,
                                              (hipStream_t)hip_stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_moments_adjoint");
}

int lbm_init_adjoint(lbm_handle* h, const float* adj, const double* rho, const double* u, double* g_rho,
                     double* g_u, void* hip_stream) {
  CHECK_HANDLE(h, "lbm_init_adjoint");
  if (h->k.aa) return fail(LBM_EINVAL, "lbm_init_adjoint: the adjoint runs on the AB layout only");
  CHECK_REQ(adj, "lbm_init_adjoint", "adj");
  CHECK_PTR(rho, "lbm_init_adjoint", "rho");
  CHECK_PTR(u, "lbm_init_adjoint", "u");
  CHECK_PTR(g_rho, "lbm_init_adjoint", "g_rho");
  CHECK_PTR(g_u, "lbm_init_adjoint", "g_u");
  hipError_t e = clbm::launch_init_adjoint(*h, adj, rho, u, g_rho, g_u, (hipStream_t)hip_stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_init_adjoint");
}

int lbm_adjoint_to_natural(lbm_handle* h, const float* slots, double* natural, void* hip_stream) {
  CHECK_HANDLE(h, "lbm_adjoint_to_natural");
  if (h->k.aa) return fail(LBM_EINVAL, "lbm_adjoint_to_natural: the adjoint runs on the AB layout only");
  CHECK_REQ(slots, "lbm_adjoint_to_natural", "slots");
  CHECK_REQ(natural, "lbm_adjoint_to_natural", "natural");
  hipError_t e = clbm::launch_adjoint_natural(*h, slots, natural, 1, nullptr, nullptr, (hipStream_t)hip_stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_adjoint_to_natural");
}

int lbm_adjoint_from_natural(lbm_handle* h, const double* natural, float* slots, void* hip_stream) {
  CHECK_HANDLE(h, "lbm_adjoint_from_natural");
  if (h->k.aa) return fail(LBM_EINVAL, "lbm_adjoint_from_natural: the adjoint runs on the AB layout only");
  CHECK_REQ(slots, "lbm_adjoint_from_natural", "slots");
  CHECK_REQ(natural, "lbm_adjoint_from_natural", "natural");
  hipError_t e = clbm::launch_adjoint_natural(*h, nullptr, nullptr, 0, natural, slots, (hipStream_t)hip_stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_adjoint_from_natural");
}

}  // extern "C"
