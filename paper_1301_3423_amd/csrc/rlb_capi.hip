// Host side of the C ABI declared in include/rlb.h.
#include "rlb.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
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

// ---- batches of shock tubes -------------------------------------------------

} // extern "C"

struct rlb_batch {
  int precision;
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

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

bool valid_tube(const rlb_tube &tb) {
  if (tb.n < 1 || tb.n > (1 << 27)) return false;
  if (tb.tau_mode == RLB_TAU_FIXED) return tb.tau > 0.5 && std::isfinite(tb.tau);
  if (tb.tau_mode == RLB_TAU_ETA_S) return tb.eta_s > 0.0 && std::isfinite(tb.eta_s);
  return false;
}

size_t batch_header_bytes(int ntubes) {
  return align256(ntubes * sizeof(rlb::TubeDesc)) + align256(ntubes * sizeof(int)) +
         align256(ntubes * sizeof(unsigned));
}

size_t tube_buffer_bytes(int32_t n, int precision) {
  return align256(static_cast<size_t>(rlb::Q) * pop_stride(n, precision) * elem_bytes(precision));
}

rlb::Geom tube_geom(const rlb_batch *b, int j) {
  rlb::Geom g;
  g.nx = 1;
  g.ny = 1;
  g.nz = b->tubes[j].n;
  g.cells = b->tubes[j].n;
  g.stride = b->desc[j].stride;
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

size_t rlb_batch_bytes(const rlb_tube *tubes, int32_t ntubes, int32_t precision) {
  if (!tubes || ntubes < 1 || (precision != RLB_FP64 && precision != RLB_MIXED)) return 0;
  size_t total = batch_header_bytes(ntubes);
  for (int j = 0; j < ntubes; ++j) {
    if (!valid_tube(tubes[j])) return 0;
    total += 2 * tube_buffer_bytes(tubes[j].n, precision);
  }
  return total;
}

int rlb_batch_create(rlb_batch **out, const rlb_tube *tubes, int32_t ntubes, int32_t precision, void *d_buf,
                     size_t bytes, void *stream) {
  if (!out || !tubes || !d_buf) return fail(RLB_EINVAL, "rlb_batch_create: NULL argument");
  *out = nullptr;
  if (ntubes < 1) return fail(RLB_EINVAL, "rlb_batch_create: no tubes");
  if (precision != RLB_FP64 && precision != RLB_MIXED) return fail(RLB_EINVAL, "rlb_batch_create: bad precision");
  for (int j = 0; j < ntubes; ++j)
    if (!valid_tube(tubes[j])) return fail(RLB_EINVAL, "rlb_batch_create: tube " + std::to_string(j) + " is invalid");
  if (reinterpret_cast<uintptr_t>(d_buf) % 256 != 0) return fail(RLB_EINVAL, "rlb_batch_create: buffer not 256-byte aligned");
  const size_t need = rlb_batch_bytes(tubes, ntubes, precision);
  if (bytes < need)
    return fail(RLB_ENOMEM, "rlb_batch_create: buffer has " + std::to_string(bytes) + " bytes, needs " + std::to_string(need));
  int dev = 0;
  RLB_HIP(hipGetDevice(&dev));
  rlb_batch *b = new (std::nothrow) rlb_batch();
  if (!b) return fail(RLB_EINVAL, "rlb_batch_create: out of host memory");
  b->precision = precision;
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
    const size_t tb = tube_buffer_bytes(tubes[j].n, precision);
    d.off[0] = static_cast<int64_t>(off / eb);
    d.off[1] = static_cast<int64_t>((off + tb) / eb);
    off += 2 * tb;
    d.steps = 0;
    d.n = tubes[j].n;
    d.stride = static_cast<int32_t>(pop_stride(tubes[j].n, precision));
    d.cur = 0;
    d.mode = tubes[j].tau_mode == RLB_TAU_ETA_S ? 1 : 0;
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
  if (b->precision == RLB_FP64)
    hipLaunchKernelGGL(rlb::k_init<double>, grid, block, 0, b->stream, dn, de, dx, dy, dz,
                       static_cast<double *>(tube_buf(b, tube, cur)), g, b->d_status + tube);
  else
    hipLaunchKernelGGL(rlb::k_init<float>, grid, block, 0, b->stream, dn, de, dx, dy, dz,
                       static_cast<float *>(tube_buf(b, tube, cur)), g, b->d_status + tube);
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
  int rc = wait_staged(b);
  if (rc != RLB_OK) return rc;
  // longest work first (cells x steps), ties by index
  std::vector<int> order;
  order.reserve(active);
  for (int j = 0; j < b->ntubes; ++j)
    if (steps[j] > 0) order.push_back(j);
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
    return static_cast<double>(b->tubes[a].n) * steps[a] > static_cast<double>(b->tubes[c].n) * steps[c];
  });
  for (int j = 0; j < b->ntubes; ++j) {
    b->desc[j].steps = steps[j];
    b->h_desc[j] = b->desc[j];
  }
  for (int k = 0; k < active; ++k) b->h_order[k] = order[k];
  RLB_HIP(hipMemcpyAsync(b->d_desc, b->h_desc, b->ntubes * sizeof(rlb::TubeDesc), hipMemcpyHostToDevice, b->stream));
  RLB_HIP(hipMemcpyAsync(b->d_order, b->h_order, active * sizeof(int), hipMemcpyHostToDevice, b->stream));
  RLB_HIP(hipEventRecord(b->staged, b->stream));
  b->staged_pending = true;
  const dim3 grid(active);
  if (b->precision == RLB_FP64)
    hipLaunchKernelGGL(rlb::k_tubes<double>, grid, dim3(rlb::TUBE_BLOCK), 0, b->stream,
                       reinterpret_cast<double *>(b->pops), b->d_desc, b->d_order, b->d_status);
  else
    hipLaunchKernelGGL(rlb::k_tubes<float>, grid, dim3(rlb::TUBE_BLOCK), 0, b->stream,
                       reinterpret_cast<float *>(b->pops), b->d_desc, b->d_order, b->d_status);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_tubes launch");
  for (int j = 0; j < b->ntubes; ++j) {
    b->desc[j].cur ^= static_cast<int32_t>(steps[j] & 1);
    b->desc[j].steps = 0;
    b->t[j] += steps[j];
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
  if (b->precision == RLB_FP64)
    hipLaunchKernelGGL(rlb::k_read<double>, grid, block, 0, b->stream,
                       static_cast<const double *>(tube_buf(b, tube, cur)), g, dn, de, dU, dP, b->d_status + tube);
  else
    hipLaunchKernelGGL(rlb::k_read<float>, grid, block, 0, b->stream,
                       static_cast<const float *>(tube_buf(b, tube, cur)), g, dn, de, dU, dP, b->d_status + tube);
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
