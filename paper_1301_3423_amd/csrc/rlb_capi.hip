// Host side of the C ABI declared in include/rlb.h.
#include "rlb.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "rlb_kernels.hpp"

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

// Elements between consecutive population arrays: the cell count rounded up
// to 256 bytes, plus 256 bytes, so that the arrays do not all start at the
// same offset modulo a large power of two.
int64_t pop_stride(int64_t cells, int precision) {
  const int64_t per = static_cast<int64_t>(PAD_BYTES / elem_bytes(precision));
  return (cells + per - 1) / per * per + per;
}

bool valid_dims(int32_t nx, int32_t ny, int32_t nz) {
  if (nx < 1 || ny < 1 || nz < 1) return false;
  const int64_t c = static_cast<int64_t>(nx) * ny * nz;
  // the kernels address (member offset + cell) * 8 bytes with 32-bit
  // unsigned offsets: (stride + cells) * 8 < 2^32 for cells <= 2^27
  return c <= (int64_t(1) << 27);
}

} // namespace

struct rlb_solver {
  rlb_config cfg;
  int device;
  hipStream_t stream;
  char *base;
  size_t bytes;
  int64_t cells;
  int64_t stride;
  size_t buf_bytes; // one population buffer
  void *buf[2];
  unsigned *status;
  int cur;
  int64_t t;
  bool initialized;
};

namespace {

rlb::Geom geom_of(const rlb_solver *s) {
  rlb::Geom g;
  g.nx = s->cfg.nx;
  g.ny = s->cfg.ny;
  g.nz = s->cfg.nz;
  g.cells = static_cast<int>(s->cells);
  g.stride = s->stride;
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

int launch_step(rlb_solver *s) {
  const rlb::Geom g = geom_of(s);
  const rlb::Relax r = relax_of(s);
  if (s->cfg.precision == RLB_FP64) {
    constexpr int TB = rlb::pair_block<double>;
    const dim3 grid(static_cast<unsigned>((s->cells + TB / 2 - 1) / (TB / 2))), block(TB);
    hipLaunchKernelGGL(rlb::k_step<double>, grid, block, 0, s->stream,
                       static_cast<const double *>(s->buf[s->cur]), static_cast<double *>(s->buf[1 - s->cur]), g, r,
                       s->status);
  } else if (s->cfg.nx % 64 == 0) {
    const dim3 grid(grid_of(s->cells)), block(rlb::BLOCK);
    hipLaunchKernelGGL(rlb::k_step_row<float>, grid, block, 0, s->stream,
                       static_cast<const float *>(s->buf[s->cur]), static_cast<float *>(s->buf[1 - s->cur]), g, r,
                       s->status);
  } else {
    constexpr int TB = rlb::pair_block<float>;
    const dim3 grid(static_cast<unsigned>((s->cells + TB / 2 - 1) / (TB / 2))), block(TB);
    hipLaunchKernelGGL(rlb::k_step<float>, grid, block, 0, s->stream,
                       static_cast<const float *>(s->buf[s->cur]), static_cast<float *>(s->buf[1 - s->cur]), g, r,
                       s->status);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_step launch");
  s->cur = 1 - s->cur;
  s->t += 1;
  return RLB_OK;
}

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

int rlb_lattice_info(rlb_lattice_t *out) {
  if (!out) return fail(RLB_EINVAL, "rlb_lattice_info: NULL");
  std::memset(out, 0, sizeof(*out));
  out->q = rlb::Q;
  out->r2 = rlb::R2;
  out->nshell = rlb::NSHELL;
  for (int i = 0; i < rlb::Q; ++i) {
    const rlb::Point &p = rlb::D3Q128[i];
    out->theta[i][0] = static_cast<int8_t>(p.tx);
    out->theta[i][1] = static_cast<int8_t>(p.ty);
    out->theta[i][2] = static_cast<int8_t>(p.tz);
    out->p0[i] = p.p0;
    out->w[i] = p.w;
    out->inv[i] = i ^ 1;
    out->shell[i] = p.shell;
  }
  static const char kSha[] =
#include "../lattice/d3q128.sha"
      ;
  std::snprintf(out->sha256, sizeof(out->sha256), "%s", kSha);
  return RLB_OK;
}

size_t rlb_state_bytes(int32_t nx, int32_t ny, int32_t nz, int32_t precision) {
  if (!valid_dims(nx, ny, nz) || (precision != RLB_FP64 && precision != RLB_MIXED)) return 0;
  const int64_t cells = static_cast<int64_t>(nx) * ny * nz;
  const size_t buf = static_cast<size_t>(rlb::Q) * pop_stride(cells, precision) * elem_bytes(precision);
  return 2 * buf + STATUS_BYTES;
}

int rlb_create(rlb_solver **out, const rlb_config *cfg, void *d_buf, size_t bytes, void *stream) {
  if (!out || !cfg || !d_buf) return fail(RLB_EINVAL, "rlb_create: NULL argument");
  *out = nullptr;
  if (!valid_dims(cfg->nx, cfg->ny, cfg->nz)) return fail(RLB_EINVAL, "rlb_create: bad lattice size");
  if (cfg->precision != RLB_FP64 && cfg->precision != RLB_MIXED)
    return fail(RLB_EINVAL, "rlb_create: bad precision");
  if (cfg->tau_mode == RLB_TAU_FIXED) {
    if (!(cfg->tau > 0.5) || !std::isfinite(cfg->tau)) return fail(RLB_EINVAL, "rlb_create: tau must exceed 1/2");
  } else if (cfg->tau_mode == RLB_TAU_ETA_S) {
    if (!(cfg->eta_s > 0.0) || !std::isfinite(cfg->eta_s)) return fail(RLB_EINVAL, "rlb_create: eta/s must be > 0");
  } else {
    return fail(RLB_EINVAL, "rlb_create: bad tau_mode");
  }
  if (reinterpret_cast<uintptr_t>(d_buf) % 256 != 0) return fail(RLB_EINVAL, "rlb_create: buffer not 256-byte aligned");
  const size_t need = rlb_state_bytes(cfg->nx, cfg->ny, cfg->nz, cfg->precision);
  if (bytes < need)
    return fail(RLB_ENOMEM, "rlb_create: buffer has " + std::to_string(bytes) + " bytes, needs " + std::to_string(need));
  int dev = 0;
  RLB_HIP(hipGetDevice(&dev));
  rlb_solver *s = new (std::nothrow) rlb_solver();
  if (!s) return fail(RLB_EINVAL, "rlb_create: out of host memory");
  s->cfg = *cfg;
  s->device = dev;
  s->stream = static_cast<hipStream_t>(stream);
  s->base = static_cast<char *>(d_buf);
  s->bytes = bytes;
  s->cells = static_cast<int64_t>(cfg->nx) * cfg->ny * cfg->nz;
  s->stride = pop_stride(s->cells, cfg->precision);
  s->buf_bytes = static_cast<size_t>(rlb::Q) * s->stride * elem_bytes(cfg->precision);
  s->buf[0] = s->base;
  s->buf[1] = s->base + s->buf_bytes;
  s->status = reinterpret_cast<unsigned *>(s->base + 2 * s->buf_bytes);
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
  // the idle buffer doubles as staging for host input (5 C doubles fit in
  // 128 C values of either precision)
  double *stage = static_cast<double *>(s->buf[1 - s->cur]);
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
  if (s->cfg.precision == RLB_FP64)
    hipLaunchKernelGGL(rlb::k_init<double>, grid, block, 0, s->stream, dn, de, dx, dy, dz,
                       static_cast<double *>(s->buf[s->cur]), g, s->status);
  else
    hipLaunchKernelGGL(rlb::k_init<float>, grid, block, 0, s->stream, dn, de, dx, dy, dz,
                       static_cast<float *>(s->buf[s->cur]), g, s->status);
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
  double *stage = static_cast<double *>(s->buf[1 - s->cur]); // 7 C doubles
  if (!on_device) {
    dn = n ? stage : nullptr;
    de = eps ? stage + C : nullptr;
    dU = U4 ? stage + 2 * C : nullptr;
    dP = P ? stage + 6 * C : nullptr;
  }
  const rlb::Geom g = geom_of(s);
  const dim3 grid(grid_of(C)), block(rlb::BLOCK);
  if (s->cfg.precision == RLB_FP64)
    hipLaunchKernelGGL(rlb::k_read<double>, grid, block, 0, s->stream, static_cast<const double *>(s->buf[s->cur]),
                       g, dn, de, dU, dP, s->status);
  else
    hipLaunchKernelGGL(rlb::k_read<float>, grid, block, 0, s->stream, static_cast<const float *>(s->buf[s->cur]),
                       g, dn, de, dU, dP, s->status);
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

int rlb_conserved(rlb_solver *s, double out[5]) {
  if (!s || !out) return fail(RLB_EINVAL, "rlb_conserved: NULL argument");
  if (!s->initialized) return fail(RLB_ESTATE, "rlb_conserved: call rlb_init_fields first");
  const rlb::Geom g = geom_of(s);
  const int chunk = rlb::BLOCK * rlb::SUM_CELLS_PER_THREAD;
  const int nblocks = static_cast<int>((s->cells + chunk - 1) / chunk);
  double *partial = static_cast<double *>(s->buf[1 - s->cur]);
  double *total = partial + static_cast<size_t>(rlb::Q) * nblocks;
  const dim3 grid1(nblocks, rlb::Q), block(rlb::BLOCK);
  if (s->cfg.precision == RLB_FP64)
    hipLaunchKernelGGL(rlb::k_popsum_partial<double>, grid1, block, 0, s->stream,
                       static_cast<const double *>(s->buf[s->cur]), g, partial, nblocks);
  else
    hipLaunchKernelGGL(rlb::k_popsum_partial<float>, grid1, block, 0, s->stream,
                       static_cast<const float *>(s->buf[s->cur]), g, partial, nblocks);
  hipLaunchKernelGGL(rlb::k_popsum_final, dim3(rlb::Q), block, 0, s->stream, partial, nblocks, total);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_popsum launch");
  double tot[rlb::Q];
  RLB_HIP(hipMemcpyAsync(tot, total, sizeof(tot), hipMemcpyDeviceToHost, s->stream));
  RLB_HIP(hipStreamSynchronize(s->stream));
  for (int k = 0; k < 5; ++k) out[k] = 0.0;
  for (int i = 0; i < rlb::Q; ++i) {
    const rlb::Point &p = rlb::D3Q128[i];
    const double pm[4] = {p.p0, p.p0 * p.tx * rlb::INV_R, p.p0 * p.ty * rlb::INV_R, p.p0 * p.tz * rlb::INV_R};
    out[0] += p.p0 * tot[i];
    for (int mu = 0; mu < 4; ++mu) out[1 + mu] += p.p0 * pm[mu] * tot[i];
  }
  return RLB_OK;
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
struct CkptHeader {
  char magic[8];
  int32_t version;
  rlb_config cfg;
  int64_t t;
  uint32_t flags;
  int32_t q;
  char sha256[65];
};
} // namespace

int rlb_save(rlb_solver *s, const char *path) {
  if (!s || !path) return fail(RLB_EINVAL, "rlb_save: NULL argument");
  if (!s->initialized) return fail(RLB_ESTATE, "rlb_save: nothing to save");
  CkptHeader h{};
  std::memcpy(h.magic, "RLBCKPT1", 8);
  h.version = 1;
  h.cfg = s->cfg;
  h.t = s->t;
  h.q = rlb::Q;
  rlb_lattice_t lat;
  rlb_lattice_info(&lat);
  std::memcpy(h.sha256, lat.sha256, sizeof(h.sha256));
  uint32_t flags = 0;
  int rc = rlb_status(s, &flags, nullptr);
  if (rc != RLB_OK) return rc;
  h.flags = flags;
  const size_t eb = elem_bytes(s->cfg.precision);
  std::vector<char> host(static_cast<size_t>(rlb::Q) * s->cells * eb);
  RLB_HIP(hipMemcpy2DAsync(host.data(), s->cells * eb, s->buf[s->cur], s->stride * eb, s->cells * eb, rlb::Q,
                           hipMemcpyDeviceToHost, s->stream));
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
  rlb_lattice_info(&lat);
  if (std::memcmp(h.magic, "RLBCKPT1", 8) != 0 || h.version != 1 || h.q != rlb::Q ||
      std::memcmp(h.sha256, lat.sha256, 64) != 0 || h.cfg.nx != s->cfg.nx || h.cfg.ny != s->cfg.ny ||
      h.cfg.nz != s->cfg.nz || h.cfg.precision != s->cfg.precision || h.cfg.tau_mode != s->cfg.tau_mode ||
      h.cfg.tau != s->cfg.tau || h.cfg.eta_s != s->cfg.eta_s) {
    std::fclose(fp);
    return fail(RLB_EINVAL, "rlb_load: checkpoint does not match this solver");
  }
  const size_t eb = elem_bytes(s->cfg.precision);
  std::vector<char> host(static_cast<size_t>(rlb::Q) * s->cells * eb);
  const bool ok = std::fread(host.data(), 1, host.size(), fp) == host.size();
  std::fclose(fp);
  if (!ok) return fail(RLB_EIO, "rlb_load: short data");
  RLB_HIP(hipMemcpy2DAsync(s->buf[s->cur], s->stride * eb, host.data(), s->cells * eb, s->cells * eb, rlb::Q,
                           hipMemcpyHostToDevice, s->stream));
  RLB_HIP(hipMemcpyAsync(s->status, &h.flags, sizeof(unsigned), hipMemcpyHostToDevice, s->stream));
  RLB_HIP(hipStreamSynchronize(s->stream));
  s->t = h.t;
  s->initialized = true;
  return RLB_OK;
}

void rlb_destroy(rlb_solver *s) { delete s; }

} // extern "C"
