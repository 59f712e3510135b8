// Host side of the C ABI declared in include/rlb.h.
#include "rlb.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <cstdlib>
#include <mutex>
#include <string>
#include <vector>

#include "rlb_kernels.hpp"

static_assert(rlb::FLAG_NONFINITE == RLB_FLAG_NONFINITE && rlb::FLAG_NONPHYSICAL == RLB_FLAG_NONPHYSICAL &&
                  rlb::FLAG_LANDAU == RLB_FLAG_LANDAU && rlb::FLAG_TUBE_SYNC == RLB_FLAG_STALL,
              "status flags of the kernels and of the C ABI must agree");

// Scratch of rlb_conserved_noalloc: the Q partial sums of every block of
// BLOCK * SUM_CELLS_PER_THREAD cells and the Q totals, for boxes of up to
// NOALLOC_MAX_BLOCKS such blocks.  One copy per GPU, held until the process
// ends (8 MiB); every call on a GPU shares it.
namespace {
constexpr int NOALLOC_MAX_BLOCKS = 8192;
constexpr int64_t NOALLOC_MAX_CELLS =
    static_cast<int64_t>(NOALLOC_MAX_BLOCKS) * rlb::BLOCK * rlb::SUM_CELLS_PER_THREAD;
constexpr size_t NOALLOC_DOUBLES = static_cast<size_t>(RLB_MAX_Q) * (NOALLOC_MAX_BLOCKS + 1);
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};
} // namespace

static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(RLB_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define RLB_HIP(call)                                                                              \
  do {                                                                                             \
    hipError_t e_ = (call);                                                                        \
    if (e_ != hipSuccess) return hip_fail(e_, #call);                                              \
  } while (0)

constexpr size_t STATUS_BYTES = 4096;
constexpr size_t PAD_BYTES = 256;

size_t elem_bytes(int precision) { return precision == RLB_MIXED ? 4 : 8; }

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// Device staging of an AA solver (it has no idle buffer): 7 doubles per
// cell for host fields, which also holds the partial sums of rlb_conserved.
size_t aa_stage_bytes(int64_t cells) { return align256(static_cast<size_t>(cells) * 7 * sizeof(double)); }

// order 0 selects the default, the third-order model
bool valid_order(int32_t o) { return o == 0 || o == RLB_ORDER2 || o == RLB_ORDER3; }
int norm_order(int32_t o) { return o == 0 ? RLB_ORDER3 : o; }
int q_of(int order) { return order == RLB_ORDER2 ? rlb::M2::Q : rlb::M3::Q; }

// Bytes of one population buffer: whole tiles of 256 / elem_bytes cells,
// each holding the Q populations of its cells in 256-byte segments (the
// tiled storage of rlb_device.hpp); a multiple of 256.
size_t pop_bytes(int64_t cells, int precision, int order) {
  const int64_t tile = static_cast<int64_t>(PAD_BYTES / elem_bytes(precision));
  const int64_t tiles = (cells + tile - 1) / tile;
  return static_cast<size_t>(tiles) * q_of(norm_order(order)) * PAD_BYTES;
}

// Calls f with a value of the model type of `order` (normalised: 2 or 3).
template <class F>
decltype(auto) with_model(int order, F &&f) {
  if (order == RLB_ORDER2) return f(rlb::M2{});
  return f(rlb::M3{});
}

bool valid_dims(int32_t nx, int32_t ny, int32_t nz) {
  if (nx < 1 || ny < 1 || nz < 1) return false;
  const int64_t c = static_cast<int64_t>(nx) * ny * nz;
  // cell indices, and the row starts the kernels form from them, stay
  // within a signed 32-bit int with a margin
  return c <= (int64_t(1) << 28) - (int64_t(1) << 16);
}

// The one-lane row kernel (float32, rows of whole wavefronts) addresses the
// x part of a tiled element with a 32-bit byte offset below nx * Q * 4.
bool row_kernel_fits(int32_t nx) { return nx % 64 == 0 && static_cast<int64_t>(nx) * rlb::M3::Q * 4 < (int64_t(1) << 31); }

} // namespace

struct rlb_solver {
  rlb_config cfg;
  int device;
  hipStream_t stream;
  char *base;
  size_t bytes;
  int64_t cells;
  size_t buf_bytes; // one population buffer
  void *buf[2];
  unsigned *status;
  int cur;
  int64_t t;
  bool initialized;
  double *stage; // device staging for host fields and sums: the idle buffer (AB) or its own area (AA)
  // solid walls (rlb_set_walls): mask and bounce-back links in caller memory
  const uint8_t *d_solid = nullptr;
  const rlb::Link *d_links = nullptr;
  int64_t nlinks = 0;
  uint64_t solid_hash = 0; // FNV-1a of the mask, 0 without walls
};

namespace {

rlb::Geom geom_of(const rlb_solver *s) {
  rlb::Geom g;
  g.nx = s->cfg.nx;
  g.ny = s->cfg.ny;
  g.nz = s->cfg.nz;
  g.cells = static_cast<int>(s->cells);
  return g;
}

rlb::Relax relax_of(const rlb_solver *s) {
  rlb::Relax r;
  r.mode = s->cfg.tau_mode == RLB_TAU_ETA_S ? 1 : 0;
  r.tau = s->cfg.tau;
  r.eta_s = s->cfg.eta_s;
  return r;
}

unsigned grid_of(int64_t cells) { return static_cast<unsigned>((cells + rlb::BLOCK - 1) / rlb::BLOCK); }

// Layout of the current state: PULL storage (two buffers), or the natural
// (even t) or swapped (odd t) state of the single AA buffer.
int access_of(const rlb_solver *s) {
  if (s->cfg.pattern != RLB_PATTERN_AA) return rlb::PULL;
  return (s->t & 1) ? rlb::AA_ODD : rlb::AA_EVEN;
}

// The step kernels of one box, with or without walls, for access AC (with
// AA the input and output buffer is the same).
template <class M, bool WALLS, int AC>
void launch_step_kernels(rlb_solver *s, const rlb::Geom &g, const rlb::Relax &r) {
  const uint8_t *solid = WALLS ? s->d_solid : nullptr;
  void *in = s->buf[s->cur];
  void *out = AC == rlb::PULL ? s->buf[1 - s->cur] : s->buf[s->cur];
  if (s->cfg.precision == RLB_FP64) {
    constexpr int TB = rlb::pair_block<M, double, AC>;
    const dim3 grid(static_cast<unsigned>((s->cells + TB / 2 - 1) / (TB / 2))), block(TB);
    rlb::k_step<M, double, WALLS, AC><<<grid, block, 0, s->stream>>>(
        static_cast<const double *>(in), static_cast<double *>(out), g, r, s->status, solid);
  } else if (row_kernel_fits(s->cfg.nx)) {
    // rows of 64 cells: x is always wide; the odd AA step rotates its stores
    // through LDS when every block holds whole rows
    constexpr int RB = rlb::step_block<AC>;
    const dim3 grid(static_cast<unsigned>((s->cells + RB - 1) / RB)), block(RB);
    if constexpr (rlb::aa_odd(AC)) {
      if (RB % s->cfg.nx == 0)
        rlb::k_step_row<M, float, WALLS, rlb::AA_ODD_ROT><<<grid, block, 0, s->stream>>>(
            static_cast<const float *>(in), static_cast<float *>(out), g, r, s->status, solid);
      else
        rlb::k_step_row<M, float, WALLS, rlb::AA_ODD><<<grid, block, 0, s->stream>>>(
            static_cast<const float *>(in), static_cast<float *>(out), g, r, s->status, solid);
    } else {
      rlb::k_step_row<M, float, WALLS, AC><<<grid, block, 0, s->stream>>>(
          static_cast<const float *>(in), static_cast<float *>(out), g, r, s->status, solid);
    }
  } else {
    constexpr int TB = rlb::pair_block<M, float, AC>;
    const dim3 grid(static_cast<unsigned>((s->cells + TB / 2 - 1) / (TB / 2))), block(TB);
    rlb::k_step<M, float, WALLS, AC><<<grid, block, 0, s->stream>>>(
        static_cast<const float *>(in), static_cast<float *>(out), g, r, s->status, solid);
  }
  if constexpr (WALLS) {
    if (s->nlinks > 0) {
      const dim3 grid(static_cast<unsigned>((s->nlinks + rlb::BLOCK - 1) / rlb::BLOCK)), block(rlb::BLOCK);
      if (s->cfg.precision == RLB_FP64)
        rlb::k_bounce<M, double><<<grid, block, 0, s->stream>>>(static_cast<double *>(s->buf[1 - s->cur]),
                                                                s->d_links, s->nlinks);
      else
        rlb::k_bounce<M, float><<<grid, block, 0, s->stream>>>(static_cast<float *>(s->buf[1 - s->cur]),
                                                               s->d_links, s->nlinks);
    }
  }
}

// float64: the two-lane kernel; float32: one lane per cell when rows are
// whole wavefronts (nx % 64 == 0), else the two-lane kernel; with walls, the
// bounce-back copies follow on the same stream.  The AA pattern alternates
// its even and odd steps in one buffer.
int launch_step(rlb_solver *s) {
  const rlb::Geom g = geom_of(s);
  const rlb::Relax r = relax_of(s);
  const int ac = access_of(s);
  with_model(s->cfg.order, [&](auto m) {
    using M = decltype(m);
    if (s->d_solid)
      launch_step_kernels<M, true, rlb::PULL>(s, g, r);
    else if (ac == rlb::AA_EVEN)
      launch_step_kernels<M, false, rlb::AA_EVEN>(s, g, r);
    else if (ac == rlb::AA_ODD && g.nx > rlb::MAXD)
      launch_step_kernels<M, false, rlb::AA_ODD_WIDE>(s, g, r);
    else if (ac == rlb::AA_ODD)
      launch_step_kernels<M, false, rlb::AA_ODD>(s, g, r);
    else
      launch_step_kernels<M, false, rlb::PULL>(s, g, r);
    return 0;
  });
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_step launch");
  if (ac == rlb::PULL) s->cur = 1 - s->cur;
  s->t += 1;
  return RLB_OK;
}

// Device staging for host fields and sums: the AA solver's own area, or the
// idle population buffer of an AB solver (large enough: 7 doubles per cell
// fit in 66 values of either precision).
double *staging(rlb_solver *s) { return s->stage ? s->stage : static_cast<double *>(s->buf[1 - s->cur]); }

bool finite_all(const double *a, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

} // namespace

extern "C" {

const char *rlb_last_error(void) { return g_last_error.c_str(); }

const char *rlb_strerror(int code) {
  switch (code) {
  case RLB_OK: return "ok";
  case RLB_EINVAL: return "invalid argument";
  case RLB_ENOMEM: return "device buffer too small";
  case RLB_ENONPHYS: return "non-physical initial field";
  case RLB_EHIP: return "HIP runtime error";
  case RLB_ESTATE: return "call out of order";
  case RLB_EIO: return "checkpoint I/O error";
  default: return "unknown error";
  }
}

int rlb_lattice_info(int32_t order, rlb_lattice_t *out) {
  if (!out) return fail(RLB_EINVAL, "rlb_lattice_info: NULL");
  if (!valid_order(order)) return fail(RLB_EINVAL, "rlb_lattice_info: order must be 0, 2 or 3");
  order = norm_order(order);
  std::memset(out, 0, sizeof(*out));
  static const char kSha3[] =
#include "../lattice/d3q128.sha"
      ;
  static const char kSha2[] =
#include "../lattice/d3q66.sha"
      ;
  return with_model(order, [&](auto m) {
    using M = decltype(m);
    out->q = M::Q;
    out->r2 = M::R2;
    out->nshell = M::NSHELL;
    for (int i = 0; i < M::Q; ++i) {
      const rlb::Point &p = M::P[i];
      out->theta[i][0] = static_cast<int8_t>(p.tx);
      out->theta[i][1] = static_cast<int8_t>(p.ty);
      out->theta[i][2] = static_cast<int8_t>(p.tz);
      out->p0[i] = p.p0;
      out->w[i] = p.w;
      out->inv[i] = i ^ 1;
      out->shell[i] = p.shell;
    }
    std::snprintf(out->sha256, sizeof(out->sha256), "%s", M::ORDER == 2 ? kSha2 : kSha3);
    return RLB_OK;
  });
}

size_t rlb_state_bytes(int32_t nx, int32_t ny, int32_t nz, int32_t precision, int32_t order, int32_t pattern) {
  if (!valid_dims(nx, ny, nz) || (precision != RLB_FP64 && precision != RLB_MIXED) || !valid_order(order)) return 0;
  if (pattern != RLB_PATTERN_AB && pattern != RLB_PATTERN_AA) return 0;
  const int64_t cells = static_cast<int64_t>(nx) * ny * nz;
  const size_t buf = pop_bytes(cells, precision, order);
  if (pattern == RLB_PATTERN_AB) return 2 * buf + STATUS_BYTES;
  return buf + STATUS_BYTES + aa_stage_bytes(cells);
}

int rlb_create(rlb_solver **out, const rlb_config *cfg, void *d_buf, size_t bytes, void *stream) {
  if (!out || !cfg || !d_buf) return fail(RLB_EINVAL, "rlb_create: NULL argument");
  *out = nullptr;
  if (!valid_dims(cfg->nx, cfg->ny, cfg->nz)) return fail(RLB_EINVAL, "rlb_create: bad lattice size");
  if (cfg->precision != RLB_FP64 && cfg->precision != RLB_MIXED)
    return fail(RLB_EINVAL, "rlb_create: bad precision");
  if (!valid_order(cfg->order)) return fail(RLB_EINVAL, "rlb_create: order must be 0, 2 or 3");
  if (cfg->pattern != RLB_PATTERN_AB && cfg->pattern != RLB_PATTERN_AA)
    return fail(RLB_EINVAL, "rlb_create: pattern must be RLB_PATTERN_AB or RLB_PATTERN_AA");
  if (cfg->tau_mode == RLB_TAU_FIXED) {
    if (!(cfg->tau > 0.5) || !std::isfinite(cfg->tau)) return fail(RLB_EINVAL, "rlb_create: tau must exceed 1/2");
  } else if (cfg->tau_mode == RLB_TAU_ETA_S) {
    if (!(cfg->eta_s > 0.0) || !std::isfinite(cfg->eta_s)) return fail(RLB_EINVAL, "rlb_create: eta/s must be > 0");
  } else {
    return fail(RLB_EINVAL, "rlb_create: bad tau_mode");
  }
  if (reinterpret_cast<uintptr_t>(d_buf) % 256 != 0) return fail(RLB_EINVAL, "rlb_create: buffer not 256-byte aligned");
  const size_t need = rlb_state_bytes(cfg->nx, cfg->ny, cfg->nz, cfg->precision, cfg->order, cfg->pattern);
  if (bytes < need)
    return fail(RLB_ENOMEM, "rlb_create: buffer has " + std::to_string(bytes) + " bytes, needs " + std::to_string(need));
  int dev = 0;
  RLB_HIP(hipGetDevice(&dev));
  rlb_solver *s = new (std::nothrow) rlb_solver();
  if (!s) return fail(RLB_EINVAL, "rlb_create: out of host memory");
  s->cfg = *cfg;
  s->cfg.order = norm_order(cfg->order);
  s->device = dev;
  s->stream = static_cast<hipStream_t>(stream);
  s->base = static_cast<char *>(d_buf);
  s->bytes = bytes;
  s->cells = static_cast<int64_t>(cfg->nx) * cfg->ny * cfg->nz;
  s->buf_bytes = pop_bytes(s->cells, cfg->precision, s->cfg.order);
  s->buf[0] = s->base;
  if (cfg->pattern == RLB_PATTERN_AA) {
    s->buf[1] = s->base; // one buffer
    s->status = reinterpret_cast<unsigned *>(s->base + s->buf_bytes);
    s->stage = reinterpret_cast<double *>(s->base + s->buf_bytes + STATUS_BYTES);
  } else {
    s->buf[1] = s->base + s->buf_bytes;
    s->status = reinterpret_cast<unsigned *>(s->base + 2 * s->buf_bytes);
    s->stage = nullptr; // the idle buffer, chosen per call
  }
  s->cur = 0;
  s->t = 0;
  s->initialized = false;
  *out = s;
  return RLB_OK;
}

int rlb_init_fields(rlb_solver *s, const double *n, const double *eps, const double *vx, const double *vy,
                    const double *vz, int32_t on_device) {
  if (!s || !n || !eps || !vx || !vy || !vz) return fail(RLB_EINVAL, "rlb_init_fields: NULL argument");
  const int64_t C = s->cells;
  const double *dn = n, *de = eps, *dx = vx, *dy = vy, *dz = vz;
  double *stage = staging(s);
  if (!on_device) {
    const double *arrs[5] = {n, eps, vx, vy, vz};
    for (auto a : arrs)
      if (!finite_all(a, C)) return fail(RLB_ENONPHYS, "rlb_init_fields: non-finite value");
    for (int64_t c = 0; c < C; ++c) {
      const double v2 = vx[c] * vx[c] + vy[c] * vy[c] + vz[c] * vz[c];
      if (!(n[c] > 0.0) || !(eps[c] > 0.0) || !(v2 < 1.0))
        return fail(RLB_ENONPHYS, "rlb_init_fields: cell " + std::to_string(c) + " has n<=0, eps<=0 or |v|>=1");
    }
    for (int k = 0; k < 5; ++k)
      RLB_HIP(hipMemcpyAsync(stage + k * C, arrs[k], C * sizeof(double), hipMemcpyHostToDevice, s->stream));
    dn = stage;
    de = stage + C;
    dx = stage + 2 * C;
    dy = stage + 3 * C;
    dz = stage + 4 * C;
  }
  RLB_HIP(hipMemsetAsync(s->status, 0, sizeof(unsigned), s->stream));
  const rlb::Geom g = geom_of(s);
  const dim3 grid(grid_of(C)), block(rlb::BLOCK);
  const int aa = s->cfg.pattern == RLB_PATTERN_AA ? 1 : 0; // t = 0: the natural AA state
  with_model(s->cfg.order, [&](auto m) {
    using M = decltype(m);
    if (s->cfg.precision == RLB_FP64)
      rlb::k_init<M, double><<<grid, block, 0, s->stream>>>(dn, de, dx, dy, dz, static_cast<double *>(s->buf[s->cur]),
                                                            g, s->status, aa);
    else
      rlb::k_init<M, float><<<grid, block, 0, s->stream>>>(dn, de, dx, dy, dz, static_cast<float *>(s->buf[s->cur]),
                                                           g, s->status, aa);
    return 0;
  });
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_init launch");
  if (!on_device) RLB_HIP(hipStreamSynchronize(s->stream));
  s->t = 0;
  s->initialized = true;
  return RLB_OK;
}

int rlb_step(rlb_solver *s, int64_t nsteps) {
  if (!s) return fail(RLB_EINVAL, "rlb_step: NULL solver");
  if (nsteps < 0) return fail(RLB_EINVAL, "rlb_step: negative step count");
  if (!s->initialized) return fail(RLB_ESTATE, "rlb_step: call rlb_init_fields first");
  for (int64_t k = 0; k < nsteps; ++k) {
    const int rc = launch_step(s);
    if (rc != RLB_OK) return rc;
  }
  return RLB_OK;
}

int rlb_read_fields(rlb_solver *s, double *n, double *eps, double *U4, double *P, int32_t on_device) {
  if (!s) return fail(RLB_EINVAL, "rlb_read_fields: NULL solver");
  if (!s->initialized) return fail(RLB_ESTATE, "rlb_read_fields: call rlb_init_fields first");
  const int64_t C = s->cells;
  double *dn = n, *de = eps, *dU = U4, *dP = P;
  double *stage = staging(s); // 7 C doubles
  if (!on_device) {
    dn = n ? stage : nullptr;
    de = eps ? stage + C : nullptr;
    dU = U4 ? stage + 2 * C : nullptr;
    dP = P ? stage + 6 * C : nullptr;
  }
  const rlb::Geom g = geom_of(s);
  const dim3 grid(grid_of(C)), block(rlb::BLOCK);
  with_model(s->cfg.order, [&](auto m) {
    using M = decltype(m);
    if (s->cfg.precision == RLB_FP64)
      rlb::k_read<M, double><<<grid, block, 0, s->stream>>>(static_cast<const double *>(s->buf[s->cur]), g, dn, de, dU,
                                                            dP, s->status, s->d_solid, access_of(s));
    else
      rlb::k_read<M, float><<<grid, block, 0, s->stream>>>(static_cast<const float *>(s->buf[s->cur]), g, dn, de, dU,
                                                           dP, s->status, s->d_solid, access_of(s));
    return 0;
  });
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_read launch");
  if (!on_device) {
    if (n) RLB_HIP(hipMemcpyAsync(n, dn, C * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    if (eps) RLB_HIP(hipMemcpyAsync(eps, de, C * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    if (U4) RLB_HIP(hipMemcpyAsync(U4, dU, 4 * C * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    if (P) RLB_HIP(hipMemcpyAsync(P, dP, C * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    RLB_HIP(hipStreamSynchronize(s->stream));
  }
  return RLB_OK;
}

namespace {
int popsum_blocks(int64_t cells) {
  const int64_t chunk = static_cast<int64_t>(rlb::BLOCK) * rlb::SUM_CELLS_PER_THREAD;
  return static_cast<int>((cells + chunk - 1) / chunk);
}

// Box totals of N^0 and T^{0 nu} from the per-population totals (streaming
// keeps each of them): k_popsum_partial writes Q * nblocks partial sums to
// `partial`, k_popsum_final the Q totals after them, in a fixed order;
// synchronises the stream.
int conserved_popsum(rlb_solver *s, double *partial, double out[5]) {
  const rlb::Geom g = geom_of(s);
  const int nblocks = popsum_blocks(s->cells);
  const int Q = q_of(s->cfg.order);
  double *total = partial + static_cast<size_t>(Q) * nblocks;
  const dim3 grid1(nblocks, Q), block(rlb::BLOCK);
  with_model(s->cfg.order, [&](auto m) {
    using M = decltype(m);
    if (s->cfg.precision == RLB_FP64)
      rlb::k_popsum_partial<M, double, true><<<grid1, block, 0, s->stream>>>(
          static_cast<const double *>(s->buf[s->cur]), g, 0, partial, nblocks);
    else
      rlb::k_popsum_partial<M, float, true><<<grid1, block, 0, s->stream>>>(
          static_cast<const float *>(s->buf[s->cur]), g, 0, partial, nblocks);
    return 0;
  });
  hipLaunchKernelGGL(rlb::k_popsum_final, dim3(Q), block, 0, s->stream, partial, nblocks, total);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_popsum launch");
  double tot[RLB_MAX_Q];
  RLB_HIP(hipMemcpyAsync(tot, total, Q * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  RLB_HIP(hipStreamSynchronize(s->stream));
  for (int k = 0; k < 5; ++k) out[k] = 0.0;
  // in the swapped AA state the values of population i sit in array inv(i)
  const int swap = access_of(s) == rlb::AA_ODD ? 1 : 0;
  with_model(s->cfg.order, [&](auto m) {
    using M = decltype(m);
    for (int i = 0; i < M::Q; ++i) {
      const rlb::Point &p = M::P[i];
      const double pm[4] = {p.p0, p.p0 * p.tx * M::INV_R, p.p0 * p.ty * M::INV_R, p.p0 * p.tz * M::INV_R};
      out[0] += p.p0 * tot[i ^ swap];
      for (int mu = 0; mu < 4; ++mu) out[1 + mu] += p.p0 * pm[mu] * tot[i ^ swap];
    }
    return 0;
  });
  return RLB_OK;
}

// Device address of the scratch array on device `dev`, looked up once per
// device with that device current (each GPU holds its own copy of the
// array; its host-side name is not a device address).
int scratch_of_device(int dev, double **out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (dev < 0 || dev >= MAX_DEVICES) return fail(RLB_EINVAL, "scratch: device index out of range");
  if (!g_scratch_ptr[dev]) {
    int cur = -1;
    RLB_HIP(hipGetDevice(&cur));
    if (cur != dev) RLB_HIP(hipSetDevice(dev));
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(RLB_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<double *>(g_scratch_ptr[dev]);
  return RLB_OK;
}
} // namespace

namespace {
// Box totals with walls: per-cell N^0 and T^{0 nu} into the idle buffer,
// then the fixed-order two-pass reduction over those five arrays.
int conserved_walls(rlb_solver *s, double out[5]) {
  const rlb::Geom g = geom_of(s);
  const int64_t C = s->cells;
  double *cellv = staging(s); // 5 C doubles
  const int chunk = rlb::BLOCK * rlb::SUM_CELLS_PER_THREAD;
  const int nblocks = static_cast<int>((C + chunk - 1) / chunk);
  double *partial = cellv + 5 * C;
  double *total = partial + 5 * static_cast<size_t>(nblocks);
  with_model(s->cfg.order, [&](auto m) {
    using M = decltype(m);
    if (s->cfg.precision == RLB_FP64)
      rlb::k_cell_conserved<M, double><<<dim3(grid_of(C)), dim3(rlb::BLOCK), 0, s->stream>>>(
          static_cast<const double *>(s->buf[s->cur]), g, s->d_solid, cellv);
    else
      rlb::k_cell_conserved<M, float><<<dim3(grid_of(C)), dim3(rlb::BLOCK), 0, s->stream>>>(
          static_cast<const float *>(s->buf[s->cur]), g, s->d_solid, cellv);
    return 0;
  });
  // five plain rows of C values
  rlb::k_popsum_partial<rlb::M3, double, false><<<dim3(nblocks, 5), dim3(rlb::BLOCK), 0, s->stream>>>(
      cellv, g, C, partial, nblocks);
  hipLaunchKernelGGL(rlb::k_popsum_final, dim3(5), dim3(rlb::BLOCK), 0, s->stream, partial, nblocks, total);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "conserved (walls) launch");
  RLB_HIP(hipMemcpyAsync(out, total, 5 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  RLB_HIP(hipStreamSynchronize(s->stream));
  return RLB_OK;
}
} // namespace

int rlb_conserved(rlb_solver *s, double out[5]) {
  if (!s || !out) return fail(RLB_EINVAL, "rlb_conserved: NULL argument");
  if (!s->initialized) return fail(RLB_ESTATE, "rlb_conserved: call rlb_init_fields first");
  if (s->d_solid) return conserved_walls(s, out);
  return conserved_popsum(s, staging(s), out);
}

int rlb_conserved_noalloc(rlb_solver *s, double out[5]) {
  if (!s || !out) return fail(RLB_EINVAL, "rlb_conserved_noalloc: NULL argument");
  if (s->d_solid)
    return fail(RLB_EINVAL, "rlb_conserved_noalloc: a box with walls needs per-cell sums; use rlb_conserved");
  if (popsum_blocks(s->cells) > NOALLOC_MAX_BLOCKS)
    return fail(RLB_EINVAL, "rlb_conserved_noalloc: " + std::to_string(s->cells) +
                                " cells exceed the fixed scratch array (at most " +
                                std::to_string(NOALLOC_MAX_CELLS) + " cells)");
  if (!s->initialized) return fail(RLB_ESTATE, "rlb_conserved_noalloc: call rlb_init_fields first");
  double *partial = nullptr;
  const int rc = scratch_of_device(s->device, &partial);
  if (rc != RLB_OK) return rc;
  return conserved_popsum(s, partial, out);
}

int rlb_status(rlb_solver *s, uint32_t *flags, int64_t *t) {
  if (!s) return fail(RLB_EINVAL, "rlb_status: NULL solver");
  if (flags) {
    unsigned h = 0;
    RLB_HIP(hipMemcpyAsync(&h, s->status, sizeof(unsigned), hipMemcpyDeviceToHost, s->stream));
    RLB_HIP(hipStreamSynchronize(s->stream));
    *flags = h;
  }
  if (t) *t = s->t;
  return RLB_OK;
}

namespace {
// version 4: the populations are stored as the library holds them on the
// device, in whole tiles (version 3 held one array per population); the
// configuration carries the model order, the header the hash of the solid
// mask (0 without walls)
constexpr int32_t CKPT_VERSION = 4;
struct CkptHeader {
  char magic[8];
  int32_t version;
  rlb_config cfg;
  int64_t t;
  uint32_t flags;
  int32_t q;
  char sha256[65];
  uint64_t solid_hash;
};
} // namespace

int rlb_save(rlb_solver *s, const char *path) {
  if (!s || !path) return fail(RLB_EINVAL, "rlb_save: NULL argument");
  if (!s->initialized) return fail(RLB_ESTATE, "rlb_save: nothing to save");
  CkptHeader h{};
  std::memcpy(h.magic, "RLBCKPT1", 8);
  h.version = CKPT_VERSION;
  h.cfg = s->cfg;
  h.t = s->t;
  h.q = q_of(s->cfg.order);
  h.solid_hash = s->solid_hash;
  rlb_lattice_t lat;
  rlb_lattice_info(s->cfg.order, &lat);
  std::memcpy(h.sha256, lat.sha256, sizeof(h.sha256));
  uint32_t flags = 0;
  int rc = rlb_status(s, &flags, nullptr);
  if (rc != RLB_OK) return rc;
  h.flags = flags;
  // the population buffer as stored: whole tiles (rlb_device.hpp)
  std::vector<char> host(s->buf_bytes);
  RLB_HIP(hipMemcpyAsync(host.data(), s->buf[s->cur], s->buf_bytes, hipMemcpyDeviceToHost, s->stream));
  RLB_HIP(hipStreamSynchronize(s->stream));
  FILE *fp = std::fopen(path, "wb");
  if (!fp) return fail(RLB_EIO, std::string("rlb_save: cannot open ") + path);
  bool ok = std::fwrite(&h, sizeof(h), 1, fp) == 1 && std::fwrite(host.data(), 1, host.size(), fp) == host.size();
  ok = (std::fclose(fp) == 0) && ok;
  if (!ok) return fail(RLB_EIO, std::string("rlb_save: short write to ") + path);
  return RLB_OK;
}

int rlb_load(rlb_solver *s, const char *path) {
  if (!s || !path) return fail(RLB_EINVAL, "rlb_load: NULL argument");
  FILE *fp = std::fopen(path, "rb");
  if (!fp) return fail(RLB_EIO, std::string("rlb_load: cannot open ") + path);
  CkptHeader h{};
  if (std::fread(&h, sizeof(h), 1, fp) != 1) {
    std::fclose(fp);
    return fail(RLB_EIO, "rlb_load: short header");
  }
  rlb_lattice_t lat;
  rlb_lattice_info(s->cfg.order, &lat);
  const int Q = q_of(s->cfg.order);
  if (std::memcmp(h.magic, "RLBCKPT1", 8) != 0 || h.version != CKPT_VERSION || h.q != Q ||
      std::memcmp(h.sha256, lat.sha256, 64) != 0 || h.cfg.nx != s->cfg.nx || h.cfg.ny != s->cfg.ny ||
      h.cfg.nz != s->cfg.nz || h.cfg.precision != s->cfg.precision || h.cfg.tau_mode != s->cfg.tau_mode ||
      h.cfg.tau != s->cfg.tau || h.cfg.eta_s != s->cfg.eta_s || h.cfg.order != s->cfg.order ||
      h.cfg.pattern != s->cfg.pattern ||
      h.solid_hash != s->solid_hash) {
    std::fclose(fp);
    return fail(RLB_EINVAL, "rlb_load: checkpoint does not match this solver");
  }
  std::vector<char> host(s->buf_bytes);
  const bool ok = std::fread(host.data(), 1, host.size(), fp) == host.size();
  std::fclose(fp);
  if (!ok) return fail(RLB_EIO, "rlb_load: short data");
  RLB_HIP(hipMemcpyAsync(s->buf[s->cur], host.data(), s->buf_bytes, hipMemcpyHostToDevice, s->stream));
  RLB_HIP(hipMemcpyAsync(s->status, &h.flags, sizeof(unsigned), hipMemcpyHostToDevice, s->stream));
  RLB_HIP(hipStreamSynchronize(s->stream));
  s->t = h.t;
  s->initialized = true;
  return RLB_OK;
}

// ---- solid walls ---------------------------------------------------------------

} // extern "C"

namespace {

uint64_t fnv1a(const uint8_t *p, int64_t n) {
  uint64_t h = 1469598103934665603ull;
  for (int64_t i = 0; i < n; ++i) {
    h ^= p[i] ? 1u : 0u; // the mask's meaning, not its byte values
    h *= 1099511628211ull;
  }
  return h ? h : 1;
}

// Bounce-back links of a mask: for every solid cell s and population i
// whose target s + theta_i is fluid, (s, s + theta_i, i); grouped by
// population, cells ascending.  Returns false if no cell is fluid.
template <class M>
bool build_links(int nx, int ny, int nz, const uint8_t *solid, std::vector<rlb::Link> *links, int64_t *count) {
  const int64_t C = static_cast<int64_t>(nx) * ny * nz;
  bool any_fluid = false;
  for (int64_t c = 0; c < C && !any_fluid; ++c) any_fluid = solid[c] == 0;
  if (!any_fluid) return false;
  int64_t n = 0;
  for (int i = 0; i < M::Q; ++i) {
    const rlb::Point &p = M::P[i];
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          const int64_t sc = x + static_cast<int64_t>(nx) * (y + static_cast<int64_t>(ny) * z);
          if (!solid[sc]) continue;
          const int xt = ((x + p.tx) % nx + nx) % nx, yt = ((y + p.ty) % ny + ny) % ny, zt = ((z + p.tz) % nz + nz) % nz;
          const int64_t tc = xt + static_cast<int64_t>(nx) * (yt + static_cast<int64_t>(ny) * zt);
          if (solid[tc]) continue;
          if (links) links->push_back(rlb::Link{static_cast<int32_t>(sc), static_cast<int32_t>(tc), i});
          ++n;
        }
  }
  *count = n;
  return true;
}

size_t walls_bytes_for(int64_t cells, int64_t nlinks) {
  return align256(static_cast<size_t>(cells)) + align256(static_cast<size_t>(nlinks) * sizeof(rlb::Link));
}

} // namespace

extern "C" {

size_t rlb_walls_bytes(int32_t order, int32_t nx, int32_t ny, int32_t nz, const uint8_t *solid) {
  if (!solid || !valid_dims(nx, ny, nz) || !valid_order(order)) return 0;
  int64_t n = 0;
  const bool ok = with_model(norm_order(order), [&](auto m) {
    using M = decltype(m);
    return build_links<M>(nx, ny, nz, solid, nullptr, &n);
  });
  if (!ok) return 0;
  return walls_bytes_for(static_cast<int64_t>(nx) * ny * nz, n);
}

int rlb_set_walls(rlb_solver *s, const uint8_t *solid, void *d_buf, size_t bytes) {
  if (!s) return fail(RLB_EINVAL, "rlb_set_walls: NULL solver");
  if (!solid) {
    s->d_solid = nullptr;
    s->d_links = nullptr;
    s->nlinks = 0;
    s->solid_hash = 0;
    return RLB_OK;
  }
  if (s->cfg.pattern == RLB_PATTERN_AA)
    return fail(RLB_EINVAL, "rlb_set_walls: walls need the AB pattern (two buffers)");
  if (!d_buf) return fail(RLB_EINVAL, "rlb_set_walls: NULL buffer");
  if (reinterpret_cast<uintptr_t>(d_buf) % 256 != 0) return fail(RLB_EINVAL, "rlb_set_walls: buffer not 256-byte aligned");
  std::vector<rlb::Link> links;
  int64_t n = 0;
  const bool ok = with_model(s->cfg.order, [&](auto m) {
    using M = decltype(m);
    return build_links<M>(s->cfg.nx, s->cfg.ny, s->cfg.nz, solid, &links, &n);
  });
  if (!ok) return fail(RLB_EINVAL, "rlb_set_walls: every cell is solid");
  const size_t need = walls_bytes_for(s->cells, n);
  if (bytes < need)
    return fail(RLB_ENOMEM, "rlb_set_walls: buffer has " + std::to_string(bytes) + " bytes, needs " + std::to_string(need));
  char *p = static_cast<char *>(d_buf);
  uint8_t *d_solid = reinterpret_cast<uint8_t *>(p);
  rlb::Link *d_links = reinterpret_cast<rlb::Link *>(p + align256(static_cast<size_t>(s->cells)));
  // the mask as 0/1 bytes
  std::vector<uint8_t> mask(static_cast<size_t>(s->cells));
  for (int64_t c = 0; c < s->cells; ++c) mask[c] = solid[c] ? 1 : 0;
  RLB_HIP(hipMemcpyAsync(d_solid, mask.data(), mask.size(), hipMemcpyHostToDevice, s->stream));
  if (n > 0)
    RLB_HIP(hipMemcpyAsync(d_links, links.data(), links.size() * sizeof(rlb::Link), hipMemcpyHostToDevice, s->stream));
  RLB_HIP(hipStreamSynchronize(s->stream));
  s->d_solid = d_solid;
  s->d_links = d_links;
  s->nlinks = n;
  s->solid_hash = fnv1a(mask.data(), s->cells);
  return RLB_OK;
}

// ---- batches of shock tubes -------------------------------------------------

} // extern "C"

struct rlb_batch {
  int precision;
  int order;
  int device;
  hipStream_t stream;
  char *base;
  size_t bytes;
  int ntubes;
  std::vector<rlb_tube> tubes;
  std::vector<rlb::TubeDesc> desc; // host view (cur, steps updated per launch)
  std::vector<int64_t> t;
  std::vector<char> initialized;
  rlb::TubeDesc *d_desc;
  int *d_order;
  unsigned *d_status;
  char *pops; // population area
  // pinned staging for descriptors and order, guarded by an event
  rlb::TubeDesc *h_desc;
  int *h_order;
  hipEvent_t staged;
  bool staged_pending;
};

namespace {

// A tube has at most 2^22 cells: the float32 tube kernel addresses its
// tiled elements with 32-bit byte offsets (below n * Q * 4).
bool valid_tube(const rlb_tube &tb) {
  if (tb.n < 1 || tb.n > (1 << 22)) return false;
  if (tb.tau_mode == RLB_TAU_FIXED) return tb.tau > 0.5 && std::isfinite(tb.tau);
  if (tb.tau_mode == RLB_TAU_ETA_S) return tb.eta_s > 0.0 && std::isfinite(tb.eta_s);
  return false;
}

// Chunks of one wavefront in the tube kernel, the most a workgroup's flags
// hold, and the most (step, chunk) items one launch gives a tube.
int64_t tube_chunks(int32_t n, int precision) {
  const int ch = precision == RLB_FP64 ? rlb::TUBE_CHUNK<double> : rlb::TUBE_CHUNK<float>;
  return (static_cast<int64_t>(n) + ch - 1) / ch;
}
int64_t tube_flow_chunks(int precision) {
  return precision == RLB_FP64 ? rlb::TUBE_FLOW_CHUNKS<double> : rlb::TUBE_FLOW_CHUNKS<float>;
}
constexpr int64_t TUBE_ITEMS_MAX = (int64_t(1) << 31) - 1;

size_t batch_header_bytes(int ntubes) {
  return align256(ntubes * sizeof(rlb::TubeDesc)) + align256(ntubes * sizeof(int)) +
         align256(ntubes * sizeof(unsigned));
}

size_t tube_buffer_bytes(int32_t n, int precision, int order) { return pop_bytes(n, precision, order); }

rlb::Geom tube_geom(const rlb_batch *b, int j) {
  rlb::Geom g;
  g.nx = 1;
  g.ny = 1;
  g.nz = b->tubes[j].n;
  g.cells = b->tubes[j].n;
  return g;
}

void *tube_buf(rlb_batch *b, int j, int which) {
  const size_t eb = elem_bytes(b->precision);
  return b->pops - 0 + static_cast<size_t>(b->desc[j].off[which]) * eb;
}

int wait_staged(rlb_batch *b) {
  if (b->staged_pending) {
    RLB_HIP(hipEventSynchronize(b->staged));
    b->staged_pending = false;
  }
  return RLB_OK;
}

} // namespace

extern "C" {

size_t rlb_batch_bytes(const rlb_tube *tubes, int32_t ntubes, int32_t precision, int32_t order) {
  if (!tubes || ntubes < 1 || (precision != RLB_FP64 && precision != RLB_MIXED) || !valid_order(order)) return 0;
  size_t total = batch_header_bytes(ntubes);
  for (int j = 0; j < ntubes; ++j) {
    if (!valid_tube(tubes[j])) return 0;
    total += 2 * tube_buffer_bytes(tubes[j].n, precision, norm_order(order));
  }
  return total;
}

int rlb_batch_create(rlb_batch **out, const rlb_tube *tubes, int32_t ntubes, int32_t precision, int32_t order,
                     void *d_buf, size_t bytes, void *stream) {
  if (!out || !tubes || !d_buf) return fail(RLB_EINVAL, "rlb_batch_create: NULL argument");
  *out = nullptr;
  if (ntubes < 1) return fail(RLB_EINVAL, "rlb_batch_create: no tubes");
  if (precision != RLB_FP64 && precision != RLB_MIXED) return fail(RLB_EINVAL, "rlb_batch_create: bad precision");
  if (!valid_order(order)) return fail(RLB_EINVAL, "rlb_batch_create: order must be 0, 2 or 3");
  order = norm_order(order);
  for (int j = 0; j < ntubes; ++j)
    if (!valid_tube(tubes[j])) return fail(RLB_EINVAL, "rlb_batch_create: tube " + std::to_string(j) + " is invalid");
  if (reinterpret_cast<uintptr_t>(d_buf) % 256 != 0) return fail(RLB_EINVAL, "rlb_batch_create: buffer not 256-byte aligned");
  const size_t need = rlb_batch_bytes(tubes, ntubes, precision, order);
  if (bytes < need)
    return fail(RLB_ENOMEM, "rlb_batch_create: buffer has " + std::to_string(bytes) + " bytes, needs " + std::to_string(need));
  int dev = 0;
  RLB_HIP(hipGetDevice(&dev));
  rlb_batch *b = new (std::nothrow) rlb_batch();
  if (!b) return fail(RLB_EINVAL, "rlb_batch_create: out of host memory");
  b->precision = precision;
  b->order = order;
  b->device = dev;
  b->stream = static_cast<hipStream_t>(stream);
  b->base = static_cast<char *>(d_buf);
  b->bytes = bytes;
  b->ntubes = ntubes;
  b->tubes.assign(tubes, tubes + ntubes);
  b->desc.resize(ntubes);
  b->t.assign(ntubes, 0);
  b->initialized.assign(ntubes, 0);
  char *p = b->base;
  b->d_desc = reinterpret_cast<rlb::TubeDesc *>(p);
  p += align256(ntubes * sizeof(rlb::TubeDesc));
  b->d_order = reinterpret_cast<int *>(p);
  p += align256(ntubes * sizeof(int));
  b->d_status = reinterpret_cast<unsigned *>(p);
  p += align256(ntubes * sizeof(unsigned));
  b->pops = p;
  const size_t eb = elem_bytes(precision);
  size_t off = 0; // bytes from pops
  for (int j = 0; j < ntubes; ++j) {
    rlb::TubeDesc &d = b->desc[j];
    const size_t tb = tube_buffer_bytes(tubes[j].n, precision, order);
    d.off[0] = static_cast<int64_t>(off / eb);
    d.off[1] = static_cast<int64_t>((off + tb) / eb);
    off += 2 * tb;
    d.steps = 0;
    d.n = tubes[j].n;
    d.cur = 0;
    d.mode = tubes[j].tau_mode == RLB_TAU_ETA_S ? 1 : 0;
    d.spin_limit = 0;
    d.tau = tubes[j].tau;
    d.eta_s = tubes[j].eta_s;
  }
  b->h_desc = nullptr;
  b->h_order = nullptr;
  b->staged_pending = false;
  hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&b->h_desc), ntubes * sizeof(rlb::TubeDesc), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&b->h_order), ntubes * sizeof(int), hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->staged, hipEventDisableTiming);
  if (e != hipSuccess) {
    if (b->h_desc) (void)hipHostFree(b->h_desc);
    if (b->h_order) (void)hipHostFree(b->h_order);
    delete b;
    return hip_fail(e, "rlb_batch_create: pinned staging");
  }
  e = hipMemsetAsync(b->d_status, 0, ntubes * sizeof(unsigned), b->stream);
  if (e != hipSuccess) {
    rlb_batch_destroy(b);
    return hip_fail(e, "rlb_batch_create: status clear");
  }
  *out = b;
  return RLB_OK;
}

int rlb_batch_init(rlb_batch *b, int32_t tube, const double *n, const double *eps, const double *vx,
                   const double *vy, const double *vz, int32_t on_device) {
  if (!b || !n || !eps || !vx || !vy || !vz) return fail(RLB_EINVAL, "rlb_batch_init: NULL argument");
  if (tube < 0 || tube >= b->ntubes) return fail(RLB_EINVAL, "rlb_batch_init: tube index out of range");
  const int64_t C = b->tubes[tube].n;
  const int cur = b->desc[tube].cur;
  const double *dn = n, *de = eps, *dx = vx, *dy = vy, *dz = vz;
  double *stage = static_cast<double *>(tube_buf(b, tube, 1 - cur));
  if (!on_device) {
    const double *arrs[5] = {n, eps, vx, vy, vz};
    for (auto a : arrs)
      if (!finite_all(a, C)) return fail(RLB_ENONPHYS, "rlb_batch_init: non-finite value");
    for (int64_t c = 0; c < C; ++c) {
      const double v2 = vx[c] * vx[c] + vy[c] * vy[c] + vz[c] * vz[c];
      if (!(n[c] > 0.0) || !(eps[c] > 0.0) || !(v2 < 1.0))
        return fail(RLB_ENONPHYS, "rlb_batch_init: cell " + std::to_string(c) + " has n<=0, eps<=0 or |v|>=1");
    }
    for (int k = 0; k < 5; ++k)
      RLB_HIP(hipMemcpyAsync(stage + k * C, arrs[k], C * sizeof(double), hipMemcpyHostToDevice, b->stream));
    dn = stage;
    de = stage + C;
    dx = stage + 2 * C;
    dy = stage + 3 * C;
    dz = stage + 4 * C;
  }
  RLB_HIP(hipMemsetAsync(b->d_status + tube, 0, sizeof(unsigned), b->stream));
  const rlb::Geom g = tube_geom(b, tube);
  const dim3 grid(grid_of(C)), block(rlb::BLOCK);
  with_model(b->order, [&](auto m) {
    using M = decltype(m);
    if (b->precision == RLB_FP64)
      rlb::k_init<M, double><<<grid, block, 0, b->stream>>>(dn, de, dx, dy, dz,
                                                            static_cast<double *>(tube_buf(b, tube, cur)), g,
                                                            b->d_status + tube, 0);
    else
      rlb::k_init<M, float><<<grid, block, 0, b->stream>>>(dn, de, dx, dy, dz,
                                                           static_cast<float *>(tube_buf(b, tube, cur)), g,
                                                           b->d_status + tube, 0);
    return 0;
  });
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_init launch");
  if (!on_device) RLB_HIP(hipStreamSynchronize(b->stream));
  b->t[tube] = 0;
  b->initialized[tube] = 1;
  return RLB_OK;
}

int rlb_batch_step(rlb_batch *b, const int64_t *steps) {
  if (!b || !steps) return fail(RLB_EINVAL, "rlb_batch_step: NULL argument");
  int active = 0;
  for (int j = 0; j < b->ntubes; ++j) {
    if (steps[j] < 0) return fail(RLB_EINVAL, "rlb_batch_step: negative step count for tube " + std::to_string(j));
    if (steps[j] > 0 && !b->initialized[j])
      return fail(RLB_ESTATE, "rlb_batch_step: tube " + std::to_string(j) + " is not initialised");
    if (steps[j] > 0) ++active;
  }
  if (active == 0) return RLB_OK;
  std::vector<int64_t> rem(steps, steps + b->ntubes);
  // tests of the stall path bound the kernel's waits to a few polls
  const char *env = std::getenv("RLB_TUBE_SPIN_LIMIT");
  const int32_t spin_limit = env ? std::max(0, std::atoi(env)) : 0;
  for (int j = 0; j < b->ntubes; ++j) b->desc[j].spin_limit = spin_limit;
  // one launch per round: each tube takes as many of its remaining steps as
  // keep its (step, chunk) items of the launch below 2^31 (a single round
  // unless a run is very long)
  for (;;) {
    std::vector<int64_t> now(b->ntubes, 0);
    std::vector<int> flow, sync;
    for (int j = 0; j < b->ntubes; ++j) {
      if (rem[j] == 0) continue;
      const int64_t nch = tube_chunks(b->tubes[j].n, b->precision);
      if (nch <= tube_flow_chunks(b->precision)) {
        now[j] = std::min<int64_t>(rem[j], TUBE_ITEMS_MAX / nch);
        flow.push_back(j);
      } else {
        now[j] = rem[j];
        sync.push_back(j);
      }
    }
    if (flow.empty() && sync.empty()) break;
    int rc = wait_staged(b);
    if (rc != RLB_OK) return rc;
    // longest work first (cells x steps), ties by index
    const auto longest = [&](int x, int y) {
      return static_cast<double>(b->tubes[x].n) * now[x] > static_cast<double>(b->tubes[y].n) * now[y];
    };
    std::stable_sort(flow.begin(), flow.end(), longest);
    std::stable_sort(sync.begin(), sync.end(), longest);
    for (int j = 0; j < b->ntubes; ++j) {
      b->desc[j].steps = now[j];
      b->h_desc[j] = b->desc[j];
    }
    int k = 0;
    for (int j : flow) b->h_order[k++] = j;
    for (int j : sync) b->h_order[k++] = j;
    RLB_HIP(hipMemcpyAsync(b->d_desc, b->h_desc, b->ntubes * sizeof(rlb::TubeDesc), hipMemcpyHostToDevice, b->stream));
    RLB_HIP(hipMemcpyAsync(b->d_order, b->h_order, k * sizeof(int), hipMemcpyHostToDevice, b->stream));
    RLB_HIP(hipEventRecord(b->staged, b->stream));
    b->staged_pending = true;
    const int nf = static_cast<int>(flow.size()), ns = static_cast<int>(sync.size());
    with_model(b->order, [&](auto m) {
      using M = decltype(m);
      if (b->precision == RLB_FP64) {
        double *pops = reinterpret_cast<double *>(b->pops);
        if (nf > 0)
          rlb::k_tubes<M, double><<<dim3(nf), dim3(rlb::TUBE_BLOCK), 0, b->stream>>>(pops, b->d_desc, b->d_order,
                                                                                     b->d_status);
        if (ns > 0)
          rlb::k_tubes_sync<M, double><<<dim3(ns), dim3(rlb::TUBE_BLOCK), 0, b->stream>>>(
              pops, b->d_desc, b->d_order + nf, b->d_status);
      } else {
        float *pops = reinterpret_cast<float *>(b->pops);
        if (nf > 0)
          rlb::k_tubes<M, float><<<dim3(nf), dim3(rlb::TUBE_BLOCK), 0, b->stream>>>(pops, b->d_desc, b->d_order,
                                                                                    b->d_status);
        if (ns > 0)
          rlb::k_tubes_sync<M, float><<<dim3(ns), dim3(rlb::TUBE_BLOCK), 0, b->stream>>>(
              pops, b->d_desc, b->d_order + nf, b->d_status);
      }
      return 0;
    });
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "k_tubes launch");
    for (int j = 0; j < b->ntubes; ++j) {
      b->desc[j].cur ^= static_cast<int32_t>(now[j] & 1);
      b->desc[j].steps = 0;
      b->t[j] += now[j];
      rem[j] -= now[j];
    }
  }
  return RLB_OK;
}

int rlb_batch_read(rlb_batch *b, int32_t tube, double *n, double *eps, double *U4, double *P, int32_t on_device) {
  if (!b) return fail(RLB_EINVAL, "rlb_batch_read: NULL batch");
  if (tube < 0 || tube >= b->ntubes) return fail(RLB_EINVAL, "rlb_batch_read: tube index out of range");
  if (!b->initialized[tube]) return fail(RLB_ESTATE, "rlb_batch_read: tube is not initialised");
  const int64_t C = b->tubes[tube].n;
  const int cur = b->desc[tube].cur;
  double *dn = n, *de = eps, *dU = U4, *dP = P;
  double *stage = static_cast<double *>(tube_buf(b, tube, 1 - cur));
  if (!on_device) {
    dn = n ? stage : nullptr;
    de = eps ? stage + C : nullptr;
    dU = U4 ? stage + 2 * C : nullptr;
    dP = P ? stage + 6 * C : nullptr;
  }
  const rlb::Geom g = tube_geom(b, tube);
  const dim3 grid(grid_of(C)), block(rlb::BLOCK);
  with_model(b->order, [&](auto m) {
    using M = decltype(m);
    if (b->precision == RLB_FP64)
      rlb::k_read<M, double><<<grid, block, 0, b->stream>>>(static_cast<const double *>(tube_buf(b, tube, cur)), g, dn,
                                                            de, dU, dP, b->d_status + tube, nullptr, rlb::PULL);
    else
      rlb::k_read<M, float><<<grid, block, 0, b->stream>>>(static_cast<const float *>(tube_buf(b, tube, cur)), g, dn,
                                                           de, dU, dP, b->d_status + tube, nullptr, rlb::PULL);
    return 0;
  });
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_read launch");
  if (!on_device) {
    if (n) RLB_HIP(hipMemcpyAsync(n, dn, C * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    if (eps) RLB_HIP(hipMemcpyAsync(eps, de, C * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    if (U4) RLB_HIP(hipMemcpyAsync(U4, dU, 4 * C * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    if (P) RLB_HIP(hipMemcpyAsync(P, dP, C * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    RLB_HIP(hipStreamSynchronize(b->stream));
  }
  return RLB_OK;
}

int rlb_batch_status(rlb_batch *b, int32_t tube, uint32_t *flags, int64_t *t) {
  if (!b) return fail(RLB_EINVAL, "rlb_batch_status: NULL batch");
  if (tube < 0 || tube >= b->ntubes) return fail(RLB_EINVAL, "rlb_batch_status: tube index out of range");
  if (flags) {
    unsigned h = 0;
    RLB_HIP(hipMemcpyAsync(&h, b->d_status + tube, sizeof(unsigned), hipMemcpyDeviceToHost, b->stream));
    RLB_HIP(hipStreamSynchronize(b->stream));
    *flags = h;
  }
  if (t) *t = b->t[tube];
  return RLB_OK;
}

void rlb_batch_destroy(rlb_batch *b) {
  if (!b) return;
  if (b->staged_pending) (void)hipEventSynchronize(b->staged);
  (void)hipEventDestroy(b->staged);
  if (b->h_desc) (void)hipHostFree(b->h_desc);
  if (b->h_order) (void)hipHostFree(b->h_order);
  delete b;
}

void rlb_destroy(rlb_solver *s) { delete s; }

} // extern "C"

// ---- serving -------------------------------------------------------------------

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

namespace {

// First-fit allocator over the caller's pool (offsets, 256-byte granules),
// coalescing neighbours on release.
class PoolAlloc {
public:
  PoolAlloc(size_t base, size_t size) { free_[base] = size; }
  bool alloc(size_t bytes, size_t &off) {
    bytes = align256(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        off = it->first;
        const size_t rem = it->second - bytes;
        free_.erase(it);
        if (rem) free_[off + bytes] = rem;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align256(bytes);
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t largest() const {
    size_t m = 0;
    for (auto &kv : free_) m = std::max(m, kv.second);
    return m;
  }

private:
  std::map<size_t, size_t> free_;
};

struct ServeReq {
  int64_t id;
  rlb_request r;
  std::vector<double> fields; // n, eps, vx, vy, vz
  double t_submit = 0, t_admit = 0;
  size_t off = 0, bytes = 0;
  int64_t remaining = 0;
  // box
  rlb_solver *box = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  int stream_idx = 0;
  // tube
  int slot = -1;
  int cur = 0;
  int64_t tube_off[2] = {0, 0};
};

// tubes are advanced per group of one precision and one model,
// group = 2 * (precision == mixed) + (order == 2); the two groups of a
// precision share a stream.  Four streams in all, one per hardware queue of
// the process (HIP's default): streams beyond that would share queues and
// run one after another (measured on the serving mix: p50/p99 0.71/3.96 s
// with eight streams, 0.64/3.70 s with these four).
constexpr int SERVE_GROUPS = 4;
constexpr int SERVE_TUBE_STREAMS = 2;
constexpr int SERVE_BOX_STREAMS = 2;
constexpr int SERVE_STREAMS = SERVE_TUBE_STREAMS + SERVE_BOX_STREAMS;

int tube_group(int precision, int order) {
  return 2 * (precision == RLB_MIXED ? 1 : 0) + (order == RLB_ORDER2 ? 1 : 0);
}
// the stream of a tube group: one per precision
int tube_stream(int group) { return group >> 1; }

int64_t request_cells(const rlb_request &r) {
  return static_cast<int64_t>(r.nx) * r.ny * r.nz;
}

// Tubes of at least this many cells run as 1 x 1 x n boxes (still on the
// tube stream of their precision): the box kernels spread a step over n / 64
// workgroups (many CUs), where the persistent tube launch gives each tube one
// CU (about 8 MLUPS in float64, so a tube of 8000 cells and 2000 steps would
// take 2 s).
constexpr int32_t TUBE_AS_BOX_CELLS = 2048;

bool runs_as_box(const rlb_request &r) { return r.kind == RLB_REQ_BOX || r.nz >= TUBE_AS_BOX_CELLS; }
// the server's tubes always fit the dataflow form of the tube kernel
static_assert(TUBE_AS_BOX_CELLS / rlb::TUBE_CHUNK<double> <= rlb::TUBE_FLOW_CHUNKS<double> &&
              TUBE_AS_BOX_CELLS / rlb::TUBE_CHUNK<float> <= rlb::TUBE_FLOW_CHUNKS<float>);

bool request_valid(const rlb_request &r, std::string &why) {
  if (r.kind != RLB_REQ_TUBE && r.kind != RLB_REQ_BOX) return why = "bad kind", false;
  if (r.kind == RLB_REQ_TUBE && (r.nx != 1 || r.ny != 1)) return why = "a tube needs nx = ny = 1", false;
  if (!valid_dims(r.nx, r.ny, r.nz)) return why = "bad lattice size", false;
  if (r.precision != RLB_FP64 && r.precision != RLB_MIXED) return why = "bad precision", false;
  if (!valid_order(r.order)) return why = "order must be 0, 2 or 3", false;
  rlb_tube tb{r.nz, r.tau_mode, r.tau, r.eta_s};
  if (!valid_tube(tb)) return why = "bad relaxation", false;
  if (r.steps < 0) return why = "negative steps", false;
  if (!r.n || !r.eps || !r.vx || !r.vy || !r.vz) return why = "NULL field", false;
  return true;
}

} // namespace

struct rlb_server {
  int device = 0;
  char *pool = nullptr;
  size_t pool_bytes = 0;
  int chunk = 0;
  int max_tubes = 0;
  size_t table_bytes = 0; // front of the pool: tube descriptors, orders, status
  PoolAlloc *alloc = nullptr;
  rlb::TubeDesc *d_desc[SERVE_GROUPS] = {};
  int *d_order[SERVE_GROUPS] = {};
  unsigned *d_status = nullptr;
  rlb::TubeDesc *h_desc[SERVE_GROUPS] = {};
  int *h_order[SERVE_GROUPS] = {};
  std::vector<int> free_slots;
  hipStream_t streams[SERVE_STREAMS] = {};
  hipEvent_t done_ev[SERVE_STREAMS] = {}; // recorded after each stream's last issued work
  bool busy[SERVE_STREAMS] = {};          // that work may still be running
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<ServeReq *> queue;
  std::vector<ServeReq *> resident;
  std::deque<rlb_completion> done;
  bool stop = false;
  int64_t next_id = 0;
  int64_t pending = 0;
  std::atomic<int64_t> rounds{0};
  std::chrono::steady_clock::time_point t0;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

size_t tube_pair_bytes(const rlb_request &r) { return 2 * tube_buffer_bytes(r.nz, r.precision, norm_order(r.order)); }

size_t request_bytes_of(const rlb_request &r) {
  if (!runs_as_box(r)) return tube_pair_bytes(r);
  return align256(rlb_state_bytes(r.nx, r.ny, r.nz, r.precision, r.order, RLB_PATTERN_AB));
}

void finish(rlb_server *sv, ServeReq *q, int rc, unsigned flags) {
  rlb_completion c;
  c.id = q->id;
  c.rc = rc;
  c.flags = flags;
  c.t_submit = q->t_submit;
  c.t_admit = q->t_admit;
  c.t_done = sv->now();
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->done.push_back(c);
    sv->pending -= 1;
  }
  sv->cv_done.notify_all();
}

void release(rlb_server *sv, ServeReq *q) {
  if (q->graph_exec) (void)hipGraphExecDestroy(q->graph_exec);
  if (q->graph) (void)hipGraphDestroy(q->graph);
  if (q->box) rlb_destroy(q->box);
  if (q->slot >= 0) sv->free_slots.push_back(q->slot);
  if (q->bytes) sv->alloc->release(q->off, q->bytes);
  delete q;
}

// Moves a queued request onto the device: allocate, initialise.
int admit(rlb_server *sv, ServeReq *q) {
  const rlb_request &r = q->r;
  const int64_t C = request_cells(r);
  const double *f = q->fields.data();
  q->t_admit = sv->now();
  q->remaining = r.steps;
  if (runs_as_box(r)) {
    rlb_config cfg{r.nx, r.ny, r.nz, r.precision, r.tau_mode, r.tau, r.eta_s, r.order, RLB_PATTERN_AB};
    int rc = rlb_create(&q->box, &cfg, sv->pool + q->off, q->bytes, sv->streams[q->stream_idx]);
    if (rc != RLB_OK) return rc;
    return rlb_init_fields(q->box, f, f + C, f + 2 * C, f + 3 * C, f + 4 * C, 0);
  }
  // tube: two buffers at q->off, staging through the second one
  const size_t eb = elem_bytes(r.precision);
  const int order = norm_order(r.order);
  const size_t tb = tube_buffer_bytes(r.nz, r.precision, order);
  q->tube_off[0] = static_cast<int64_t>(q->off / eb);
  q->tube_off[1] = static_cast<int64_t>((q->off + tb) / eb);
  q->cur = 0;
  hipStream_t st = sv->streams[tube_stream(tube_group(r.precision, order))];
  double *stage = reinterpret_cast<double *>(sv->pool + q->off + tb);
  RLB_HIP(hipMemcpyAsync(stage, f, 5 * C * sizeof(double), hipMemcpyHostToDevice, st));
  RLB_HIP(hipMemsetAsync(sv->d_status + q->slot, 0, sizeof(unsigned), st));
  rlb::Geom g;
  g.nx = 1;
  g.ny = 1;
  g.nz = r.nz;
  g.cells = r.nz;
  const dim3 grid(grid_of(C)), block(rlb::BLOCK);
  with_model(order, [&](auto m) {
    using M = decltype(m);
    if (r.precision == RLB_FP64)
      rlb::k_init<M, double><<<grid, block, 0, st>>>(stage, stage + C, stage + 2 * C, stage + 3 * C, stage + 4 * C,
                                                     reinterpret_cast<double *>(sv->pool + q->off), g,
                                                     sv->d_status + q->slot, 0);
    else
      rlb::k_init<M, float><<<grid, block, 0, st>>>(stage, stage + C, stage + 2 * C, stage + 3 * C, stage + 4 * C,
                                                    reinterpret_cast<float *>(sv->pool + q->off), g,
                                                    sv->d_status + q->slot, 0);
    return 0;
  });
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "serve k_init");
  RLB_HIP(hipStreamSynchronize(st)); // the staged fields are consumed before the next round reuses the buffer
  return RLB_OK;
}

// Reads a finished request's fields into its host outputs; returns rc.
int complete(rlb_server *sv, ServeReq *q, unsigned &flags) {
  const rlb_request &r = q->r;
  if (runs_as_box(r)) {
    int rc = rlb_read_fields(q->box, r.out_n, r.out_eps, r.out_U4, r.out_P, 0);
    if (rc != RLB_OK) return rc;
    return rlb_status(q->box, &flags, nullptr);
  }
  const int64_t C = r.nz;
  const size_t eb = elem_bytes(r.precision);
  const int order = norm_order(r.order);
  hipStream_t st = sv->streams[tube_stream(tube_group(r.precision, order))];
  double *stage = reinterpret_cast<double *>(sv->pool + static_cast<size_t>(q->tube_off[1 - q->cur]) * eb);
  char *curp = sv->pool + static_cast<size_t>(q->tube_off[q->cur]) * eb;
  rlb::Geom g;
  g.nx = 1;
  g.ny = 1;
  g.nz = r.nz;
  g.cells = r.nz;
  const dim3 grid(grid_of(C)), block(rlb::BLOCK);
  double *dn = stage, *de = stage + C, *dU = stage + 2 * C, *dP = stage + 6 * C;
  with_model(order, [&](auto m) {
    using M = decltype(m);
    if (r.precision == RLB_FP64)
      rlb::k_read<M, double><<<grid, block, 0, st>>>(reinterpret_cast<const double *>(curp), g, dn, de, dU, dP,
                                                     sv->d_status + q->slot, nullptr, rlb::PULL);
    else
      rlb::k_read<M, float><<<grid, block, 0, st>>>(reinterpret_cast<const float *>(curp), g, dn, de, dU, dP,
                                                    sv->d_status + q->slot, nullptr, rlb::PULL);
    return 0;
  });
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "serve k_read");
  if (r.out_n) RLB_HIP(hipMemcpyAsync(r.out_n, dn, C * sizeof(double), hipMemcpyDeviceToHost, st));
  if (r.out_eps) RLB_HIP(hipMemcpyAsync(r.out_eps, de, C * sizeof(double), hipMemcpyDeviceToHost, st));
  if (r.out_U4) RLB_HIP(hipMemcpyAsync(r.out_U4, dU, 4 * C * sizeof(double), hipMemcpyDeviceToHost, st));
  if (r.out_P) RLB_HIP(hipMemcpyAsync(r.out_P, dP, C * sizeof(double), hipMemcpyDeviceToHost, st));
  unsigned h = 0;
  RLB_HIP(hipMemcpyAsync(&h, sv->d_status + q->slot, sizeof(unsigned), hipMemcpyDeviceToHost, st));
  RLB_HIP(hipStreamSynchronize(st));
  flags = h;
  return RLB_OK;
}

// Advances one box by `steps`: each full chunk replays the box's captured
// graph of `chunk` step launches, the rest is launched directly.
int box_advance(rlb_server *sv, ServeReq *q, int64_t steps) {
  hipStream_t st = sv->streams[q->stream_idx];
  int64_t full = steps / sv->chunk;
  if (full > 0 && !q->graph_exec) {
    RLB_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const int64_t t_before = q->box->t;
    const int cur_before = q->box->cur;
    int rc = rlb_step(q->box, sv->chunk);
    hipGraph_t gr = nullptr;
    hipError_t e = hipStreamEndCapture(st, &gr);
    q->box->t = t_before; // capture issued nothing: undo the host bookkeeping
    q->box->cur = cur_before;
    if (rc != RLB_OK) return rc;
    if (e != hipSuccess) return hip_fail(e, "serve graph capture");
    q->graph = gr;
    RLB_HIP(hipGraphInstantiate(&q->graph_exec, gr, nullptr, nullptr, 0));
  }
  for (; full > 0; --full) {
    RLB_HIP(hipGraphLaunch(q->graph_exec, st));
    q->box->t += sv->chunk; // chunk is even: the current buffer is unchanged
  }
  return rlb_step(q->box, steps % sv->chunk);
}

// Steps a resident box takes per issue on its stream: BOX_ISSUE_CHUNKS
// chunks for boxes of BOX_ROUND_CELLS cells or more, proportionally more (in
// whole chunks) for smaller boxes; a long tube run as a box takes
// max(1, BOX_ROUND_CELLS / n) chunks of its n cells.  Long issues keep a
// box from being interleaved with every box that arrives during its run (a
// box stream then works almost first come, first served; the two box
// streams take boxes by least work left).  On the serving mix at a fixed
// 22.3 requests/s with 50-step chunks, the p99 latency was 2.98-3.07 s with
// box issues of 1 chunk, 2.06 s with 5, 2.06-2.09 s with 10, 1.83-2.04 s with
// 20 and 1.82 s with 40 (boxes 3.3-3.6, 2.5-2.6, 2.4, 2.05-2.24 and 2.05 s;
// tubes 0.44-0.54 s; p50 0.07 s throughout).  With 40 chunks of 50 steps
// every box of that mix (at most 1000 steps) runs to the end in one issue.
// Tube rounds stay at one chunk: 1000-step tube rounds raised the tubes'
// p99 to 0.6 s.
constexpr int64_t BOX_ROUND_CELLS = 262144; // 64^3
constexpr int64_t BOX_ISSUE_CHUNKS = 40;

int64_t box_round_steps(const rlb_server *sv, const ServeReq *q) {
  int64_t chunks = std::max<int64_t>(1, BOX_ROUND_CELLS / std::max<int64_t>(request_cells(q->r), 1));
  if (q->r.kind == RLB_REQ_BOX) chunks *= BOX_ISSUE_CHUNKS;
  return std::min<int64_t>(q->remaining, chunks * sv->chunk);
}

// Steps a resident tube takes per launch of its group: at least chunk, and
// as many as fit in chunk * TUBE_ROUND_CELLS lattice updates, so short tubes
// finish in few launches while a launch stays about as long as a box chunk.
// (Measured on the serving mix at 18.4 requests/s, with all streams then
// synchronised after every launch: 4096 gave p50/p99 0.79/4.7 s, 8192
// 0.70/3.8-3.9 s, 16384 0.76/3.5 s with slower boxes.)
constexpr int64_t TUBE_ROUND_CELLS = 8192;

int64_t tube_round_steps(const rlb_server *sv, const ServeReq *q) {
  const int64_t budget = static_cast<int64_t>(sv->chunk) * TUBE_ROUND_CELLS / std::max<int64_t>(q->r.nz, 1);
  // the tube kernel counts a launch's (step, chunk) items in 32 bits
  const int64_t cap = TUBE_ITEMS_MAX / tube_chunks(q->r.nz, q->r.precision);
  return std::min<int64_t>(std::min<int64_t>(q->remaining, cap), std::max<int64_t>(sv->chunk, budget));
}

int tubes_advance(rlb_server *sv, int prec, int order, bool &issued) {
  // all resident tubes of this precision and model, one persistent launch
  std::vector<ServeReq *> tubes;
  for (ServeReq *q : sv->resident)
    if (!runs_as_box(q->r) && q->r.precision == prec && norm_order(q->r.order) == order && q->remaining > 0)
      tubes.push_back(q);
  if (tubes.empty()) return RLB_OK;
  issued = true;
  const int p = tube_group(prec, order);
  std::stable_sort(tubes.begin(), tubes.end(), [&](ServeReq *a, ServeReq *b) {
    return static_cast<double>(a->r.nz) * tube_round_steps(sv, a) >
           static_cast<double>(b->r.nz) * tube_round_steps(sv, b);
  });
  int k = 0;
  for (ServeReq *q : tubes) {
    rlb::TubeDesc &d = sv->h_desc[p][q->slot];
    d.off[0] = q->tube_off[0];
    d.off[1] = q->tube_off[1];
    d.steps = tube_round_steps(sv, q);
    d.n = q->r.nz;
    d.cur = q->cur;
    d.mode = q->r.tau_mode == RLB_TAU_ETA_S ? 1 : 0;
    d.spin_limit = 0;
    d.tau = q->r.tau;
    d.eta_s = q->r.eta_s;
    sv->h_order[p][k++] = q->slot;
  }
  hipStream_t st = sv->streams[tube_stream(p)];
  RLB_HIP(hipMemcpyAsync(sv->d_desc[p], sv->h_desc[p], sv->max_tubes * sizeof(rlb::TubeDesc), hipMemcpyHostToDevice, st));
  RLB_HIP(hipMemcpyAsync(sv->d_order[p], sv->h_order[p], k * sizeof(int), hipMemcpyHostToDevice, st));
  with_model(order, [&](auto m) {
    using M = decltype(m);
    if (prec == RLB_FP64)
      rlb::k_tubes<M, double><<<dim3(k), dim3(rlb::TUBE_BLOCK), 0, st>>>(reinterpret_cast<double *>(sv->pool),
                                                                          sv->d_desc[p], sv->d_order[p], sv->d_status);
    else
      rlb::k_tubes<M, float><<<dim3(k), dim3(rlb::TUBE_BLOCK), 0, st>>>(reinterpret_cast<float *>(sv->pool),
                                                                         sv->d_desc[p], sv->d_order[p], sv->d_status);
    return 0;
  });
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "serve k_tubes");
  for (ServeReq *q : tubes) {
    const int64_t s = tube_round_steps(sv, q);
    q->cur ^= static_cast<int>(s & 1);
    q->remaining -= s;
  }
  return RLB_OK;
}

// Population bytes a box still has to stream (read and write) in `steps` steps.
double box_bytes_left(const rlb_request &r, int64_t steps) {
  return 2.0 * static_cast<double>(steps) * static_cast<double>(request_cells(r)) * q_of(norm_order(r.order)) *
         static_cast<double>(elem_bytes(r.precision));
}

// The stream a resident request's work runs on.
int request_stream(const ServeReq *q) { return q->stream_idx; }

// The worker.  Each stream runs on its own: whenever a stream has finished
// the work last issued to it, its finished requests are read back and
// released, queued requests that go to it are admitted, and its next work
// is issued (one persistent launch per tube group of its precision, or
// `chunk` steps of each of its boxes).  No stream waits for another.
void serve_loop(rlb_server *sv) {
  (void)hipSetDevice(sv->device);
  for (;;) {
    bool any_busy = false;
    for (int i = 0; i < SERVE_STREAMS; ++i) {
      if (sv->busy[i] && hipEventQuery(sv->done_ev[i]) == hipSuccess) sv->busy[i] = false;
      any_busy = any_busy || sv->busy[i];
    }
    bool progressed = false;
    // completions on idle streams
    {
      std::vector<ServeReq *> keep;
      for (ServeReq *q : sv->resident) {
        if (q->remaining > 0 || sv->busy[request_stream(q)]) {
          keep.push_back(q);
          continue;
        }
        unsigned flags = 0;
        const int crc = complete(sv, q, flags);
        finish(sv, q, crc, flags);
        std::lock_guard<std::mutex> lk(sv->mu);
        release(sv, q);
        progressed = true;
      }
      sv->resident.swap(keep);
    }
    // admission in arrival order, while memory and tube slots allow.  A box
    // goes to the box stream with the least work left (population bytes
    // still to stream) and waits until that stream is idle; a request that
    // waits for its stream lets later requests bound for idle streams pass,
    // while one that does not fit in memory holds back all behind it.
    // (Measured on the serving mix at 21.2 requests/s against filling
    // whichever box stream was idle, in arrival order: p99 3.55 s instead of
    // 3.7-4.4 s, p50 0.32 s against 0.32-0.34 s.)
    std::vector<ServeReq *> admitted;
    double box_work[SERVE_BOX_STREAMS] = {};
    for (ServeReq *q : sv->resident)
      if (q->r.kind == RLB_REQ_BOX) box_work[q->stream_idx - SERVE_TUBE_STREAMS] += box_bytes_left(q->r, q->remaining);
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      if (sv->resident.empty() && !any_busy)
        sv->cv_work.wait(lk, [&] { return sv->stop || !sv->queue.empty(); });
      if (sv->stop) return;
      for (auto it = sv->queue.begin(); it != sv->queue.end();) {
        ServeReq *q = *it;
        int st = -1;
        if (q->r.kind == RLB_REQ_TUBE) {
          st = tube_stream(tube_group(q->r.precision, norm_order(q->r.order)));
          if (sv->busy[st] || (!runs_as_box(q->r) && sv->free_slots.empty())) st = -1;
        } else {
          // the box stream with the least work left; the box waits for it
          int best = 0;
          for (int b = 1; b < SERVE_BOX_STREAMS; ++b)
            if (box_work[b] < box_work[best] ||
                (box_work[b] == box_work[best] && sv->busy[SERVE_TUBE_STREAMS + best] && !sv->busy[SERVE_TUBE_STREAMS + b]))
              best = b;
          if (!sv->busy[SERVE_TUBE_STREAMS + best]) st = SERVE_TUBE_STREAMS + best;
        }
        if (st < 0) { // waits for its stream: later requests for idle streams go first
          ++it;
          continue;
        }
        size_t off = 0;
        if (!sv->alloc->alloc(q->bytes, off)) break;
        q->off = off;
        q->stream_idx = st;
        if (!runs_as_box(q->r)) {
          q->slot = sv->free_slots.back();
          sv->free_slots.pop_back();
        } else if (q->r.kind == RLB_REQ_BOX) {
          box_work[st - SERVE_TUBE_STREAMS] += box_bytes_left(q->r, q->r.steps);
        }
        it = sv->queue.erase(it);
        admitted.push_back(q);
      }
    }
    for (ServeReq *q : admitted) {
      progressed = true;
      const int rc = admit(sv, q);
      if (rc != RLB_OK) {
        finish(sv, q, rc, 0);
        std::lock_guard<std::mutex> lk(sv->mu);
        release(sv, q);
        continue;
      }
      sv->resident.push_back(q);
    }
    // next work on every idle stream
    for (int st = 0; st < SERVE_STREAMS; ++st) {
      if (sv->busy[st]) continue;
      int rc = RLB_OK;
      bool issued = false;
      if (st < SERVE_TUBE_STREAMS) {
        const int prec = st == tube_stream(tube_group(RLB_FP64, RLB_ORDER3)) ? RLB_FP64 : RLB_MIXED;
        for (int order : {RLB_ORDER3, RLB_ORDER2})
          if (rc == RLB_OK) rc = tubes_advance(sv, prec, order, issued);
      }
      // boxes, and on the tube streams the long tubes that run as boxes
      for (ServeReq *q : sv->resident) {
        if (rc != RLB_OK) break;
        if (!runs_as_box(q->r) || q->stream_idx != st || q->remaining == 0) continue;
        const int64_t n = box_round_steps(sv, q);
        rc = box_advance(sv, q, n);
        q->remaining -= n;
        issued = true;
      }
      if (rc != RLB_OK) {
        // a launch on this stream failed: end every request on it with the error
        (void)hipStreamSynchronize(sv->streams[st]);
        std::vector<ServeReq *> keep;
        for (ServeReq *q : sv->resident) {
          if (request_stream(q) != st) {
            keep.push_back(q);
            continue;
          }
          finish(sv, q, rc, 0);
          std::lock_guard<std::mutex> lk(sv->mu);
          release(sv, q);
        }
        sv->resident.swap(keep);
        progressed = true;
        continue;
      }
      if (issued) {
        if (hipEventRecord(sv->done_ev[st], sv->streams[st]) != hipSuccess) (void)hipStreamSynchronize(sv->streams[st]);
        else sv->busy[st] = true;
        sv->rounds += 1;
        progressed = true;
      }
    }
    if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
}

} // namespace

extern "C" {

size_t rlb_request_bytes(const rlb_request *req) {
  if (!req) return 0;
  std::string why;
  if (!request_valid(*req, why)) return 0;
  return request_bytes_of(*req);
}

int rlb_server_create(rlb_server **out, void *d_pool, size_t pool_bytes, int32_t chunk_steps, int32_t max_tubes) {
  if (!out || !d_pool) return fail(RLB_EINVAL, "rlb_server_create: NULL argument");
  *out = nullptr;
  if (chunk_steps < 2 || chunk_steps % 2) return fail(RLB_EINVAL, "rlb_server_create: chunk_steps must be even and >= 2");
  if (max_tubes < 1) return fail(RLB_EINVAL, "rlb_server_create: max_tubes must be >= 1");
  if (reinterpret_cast<uintptr_t>(d_pool) % 256 != 0) return fail(RLB_EINVAL, "rlb_server_create: pool not 256-byte aligned");
  const size_t table = SERVE_GROUPS * (align256(max_tubes * sizeof(rlb::TubeDesc)) + align256(max_tubes * sizeof(int))) +
                       align256(max_tubes * sizeof(unsigned));
  if (pool_bytes <= table) return fail(RLB_ENOMEM, "rlb_server_create: pool too small");
  int dev = 0;
  RLB_HIP(hipGetDevice(&dev));
  rlb_server *sv = new (std::nothrow) rlb_server();
  if (!sv) return fail(RLB_EINVAL, "rlb_server_create: out of host memory");
  sv->device = dev;
  sv->pool = static_cast<char *>(d_pool);
  sv->pool_bytes = pool_bytes;
  sv->chunk = chunk_steps;
  sv->max_tubes = max_tubes;
  sv->table_bytes = table;
  char *p = sv->pool;
  for (int k = 0; k < SERVE_GROUPS; ++k) {
    sv->d_desc[k] = reinterpret_cast<rlb::TubeDesc *>(p);
    p += align256(max_tubes * sizeof(rlb::TubeDesc));
    sv->d_order[k] = reinterpret_cast<int *>(p);
    p += align256(max_tubes * sizeof(int));
  }
  sv->d_status = reinterpret_cast<unsigned *>(p);
  // requests are placed after the tables; allocator offsets are from the pool start
  sv->alloc = new PoolAlloc(table, pool_bytes - table);
  for (int k = 0; k < SERVE_GROUPS; ++k) {
    hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&sv->h_desc[k]), max_tubes * sizeof(rlb::TubeDesc), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&sv->h_order[k]), max_tubes * sizeof(int), hipHostMallocDefault);
    if (e != hipSuccess) {
      rlb_server_destroy(sv);
      return hip_fail(e, "rlb_server_create: pinned tables");
    }
    std::memset(sv->h_desc[k], 0, max_tubes * sizeof(rlb::TubeDesc));
  }
  for (int i = 0; i < SERVE_STREAMS; ++i) {
    hipError_t e = hipStreamCreateWithFlags(&sv->streams[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sv->done_ev[i], hipEventDisableTiming);
    if (e != hipSuccess) {
      rlb_server_destroy(sv);
      return hip_fail(e, "rlb_server_create: streams");
    }
  }
  for (int j = max_tubes - 1; j >= 0; --j) sv->free_slots.push_back(j);
  sv->t0 = std::chrono::steady_clock::now();
  sv->worker = std::thread(serve_loop, sv);
  *out = sv;
  return RLB_OK;
}

int rlb_server_submit(rlb_server *sv, const rlb_request *req, int64_t *id) {
  if (!sv || !req) return fail(RLB_EINVAL, "rlb_server_submit: NULL argument");
  std::string why;
  if (!request_valid(*req, why)) return fail(RLB_EINVAL, "rlb_server_submit: " + why);
  const int64_t C = request_cells(*req);
  const double *arrs[5] = {req->n, req->eps, req->vx, req->vy, req->vz};
  for (auto a : arrs)
    if (!finite_all(a, C)) return fail(RLB_ENONPHYS, "rlb_server_submit: non-finite value");
  for (int64_t c = 0; c < C; ++c) {
    const double v2 = req->vx[c] * req->vx[c] + req->vy[c] * req->vy[c] + req->vz[c] * req->vz[c];
    if (!(req->n[c] > 0.0) || !(req->eps[c] > 0.0) || !(v2 < 1.0))
      return fail(RLB_ENONPHYS, "rlb_server_submit: cell " + std::to_string(c) + " has n<=0, eps<=0 or |v|>=1");
  }
  const size_t bytes = request_bytes_of(*req);
  if (bytes > sv->pool_bytes - sv->table_bytes) return fail(RLB_ENOMEM, "rlb_server_submit: request can never fit in the pool");
  ServeReq *q = new (std::nothrow) ServeReq();
  if (!q) return fail(RLB_EINVAL, "rlb_server_submit: out of host memory");
  q->r = *req;
  q->fields.resize(5 * C);
  for (int k = 0; k < 5; ++k) std::memcpy(q->fields.data() + k * C, arrs[k], C * sizeof(double));
  q->r.n = q->r.eps = q->r.vx = q->r.vy = q->r.vz = nullptr;
  q->bytes = bytes;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    q->id = sv->next_id++;
    q->t_submit = sv->now();
    sv->queue.push_back(q);
    sv->pending += 1;
  }
  sv->cv_work.notify_all();
  if (id) *id = q->id;
  return RLB_OK;
}

int rlb_server_poll(rlb_server *sv, rlb_completion *out, int32_t max, int32_t *count, int32_t wait_ms) {
  if (!sv || !out || !count || max < 1) return fail(RLB_EINVAL, "rlb_server_poll: bad argument");
  std::unique_lock<std::mutex> lk(sv->mu);
  if (sv->done.empty() && wait_ms > 0)
    sv->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !sv->done.empty(); });
  int n = 0;
  while (n < max && !sv->done.empty()) {
    out[n++] = sv->done.front();
    sv->done.pop_front();
  }
  *count = n;
  return RLB_OK;
}

int rlb_server_pending(rlb_server *sv, int64_t *pending, int64_t *rounds) {
  if (!sv) return fail(RLB_EINVAL, "rlb_server_pending: NULL server");
  std::lock_guard<std::mutex> lk(sv->mu);
  if (pending) *pending = sv->pending;
  if (rounds) *rounds = sv->rounds.load();
  return RLB_OK;
}

void rlb_server_destroy(rlb_server *sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv_work.notify_all();
  if (sv->worker.joinable()) sv->worker.join();
  for (int i = 0; i < SERVE_STREAMS; ++i)
    if (sv->streams[i]) (void)hipStreamSynchronize(sv->streams[i]);
  for (ServeReq *q : sv->resident) release(sv, q);
  for (ServeReq *q : sv->queue) {
    q->bytes = 0;
    q->slot = -1;
    release(sv, q);
  }
  for (int i = 0; i < SERVE_STREAMS; ++i) {
    if (sv->done_ev[i]) (void)hipEventDestroy(sv->done_ev[i]);
    if (sv->streams[i]) (void)hipStreamDestroy(sv->streams[i]);
  }
  for (int k = 0; k < SERVE_GROUPS; ++k) {
    if (sv->h_desc[k]) (void)hipHostFree(sv->h_desc[k]);
    if (sv->h_order[k]) (void)hipHostFree(sv->h_order[k]);
  }
  delete sv->alloc;
  delete sv;
}

} // extern "C"
