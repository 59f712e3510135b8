// Exercises every C-ABI entry point (boxes with both streaming patterns,
// walls, checkpoints, the tube batch, the server, error paths) for a build of
// the library whose host code carries AddressSanitizer and UBSan.
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <unistd.h>
#include <vector>
#include "rlb.h"
#define OK(x) do { int rc_ = (x); if (rc_ != RLB_OK) { printf("FAIL %s -> %d (%s)\n", #x, rc_, rlb_last_error()); return 1; } } while (0)
#define EXPECT(c) do { if (!(c)) { printf("FAIL expect %s line %d\n", #c, __LINE__); return 1; } } while (0)

static void fields(int nx, int ny, int nz, std::vector<double> *f) {
  const size_t C = (size_t)nx * ny * nz;
  for (int k = 0; k < 5; ++k) f[k].assign(C, 0.0);
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const size_t c = ((size_t)z * ny + y) * nx + x;
        const double T = 1.0 + 0.05 * std::sin(0.3 * x + 0.2 * y + 0.1 * z);
        f[0][c] = T * T * T;
        f[1][c] = 3.0 * T * T * T * T;
        f[2][c] = 0.2 * std::sin(0.4 * z);
        f[3][c] = 0.1 * std::cos(0.3 * x);
        f[4][c] = 0.1 * std::sin(0.5 * y);
      }
}

static int box(int order, int precision, int pattern, bool walls) {
  const int nx = 24, ny = 20, nz = 16;
  const size_t C = (size_t)nx * ny * nz;
  rlb_config cfg{nx, ny, nz, precision, RLB_TAU_ETA_S, 0.0, 0.2, order, pattern};
  const size_t bytes = rlb_state_bytes(nx, ny, nz, precision, order, pattern);
  EXPECT(bytes > 0);
  void *d = nullptr;
  if (hipMalloc(&d, bytes) != hipSuccess) return 1;
  rlb_solver *s = nullptr;
  OK(rlb_create(&s, &cfg, d, bytes, nullptr));
  std::vector<double> f[5];
  fields(nx, ny, nz, f);
  void *dw = nullptr;
  if (walls) {
    std::vector<uint8_t> solid(C, 0);
    for (int z = 0; z < nz; ++z)
      for (int x = 0; x < nx; ++x)
        for (int y = 0; y < ny; ++y)
          if (y < 6) solid[((size_t)z * ny + y) * nx + x] = 1;
    const size_t wb = rlb_walls_bytes(order, nx, ny, nz, solid.data());
    EXPECT(wb > 0);
    if (hipMalloc(&dw, wb) != hipSuccess) return 1;
    OK(rlb_set_walls(s, solid.data(), dw, wb));
  }
  OK(rlb_init_fields(s, f[0].data(), f[1].data(), f[2].data(), f[3].data(), f[4].data(), 0));
  double c0[5], c1[5];
  OK(rlb_conserved(s, c0));
  OK(rlb_step(s, 3));
  OK(rlb_conserved(s, c1));
  EXPECT(std::fabs(c1[0] - c0[0]) < 1e-6 * std::fabs(c0[0]));
  if (!walls) {
    double c2[5];
    OK(rlb_conserved_noalloc(s, c2));
    for (int k = 0; k < 5; ++k) EXPECT(c2[k] == c1[k]);
  } else {
    double c2[5];
    EXPECT(rlb_conserved_noalloc(s, c2) == RLB_EINVAL);
  }
  std::vector<double> n(C), eps(C), U(4 * C), P(C);
  OK(rlb_read_fields(s, n.data(), eps.data(), U.data(), P.data(), 0));
  uint32_t flags = 0;
  int64_t t = 0;
  OK(rlb_status(s, &flags, &t));
  EXPECT(flags == 0 && t == 3);
  if (!walls) {
    OK(rlb_save(s, "/tmp/rlb_asan.ckpt"));
    OK(rlb_step(s, 2));
    OK(rlb_load(s, "/tmp/rlb_asan.ckpt"));
    OK(rlb_status(s, &flags, &t));
    EXPECT(t == 3);
  }
  rlb_destroy(s);
  if (dw) (void)hipFree(dw);
  (void)hipFree(d);
  printf("box order %d precision %d pattern %d walls %d ok\n", order, precision, pattern, (int)walls);
  return 0;
}

static int batch(int order, int precision) {
  rlb_tube tubes[3] = {{200, RLB_TAU_ETA_S, 0.0, 0.1}, {57, RLB_TAU_FIXED, 0.9, 0.0}, {700, RLB_TAU_ETA_S, 0.0, 0.3}};
  const size_t bytes = rlb_batch_bytes(tubes, 3, precision, order);
  EXPECT(bytes > 0);
  void *d = nullptr;
  if (hipMalloc(&d, bytes) != hipSuccess) return 1;
  rlb_batch *b = nullptr;
  OK(rlb_batch_create(&b, tubes, 3, precision, order, d, bytes, nullptr));
  for (int j = 0; j < 3; ++j) {
    const int n = tubes[j].n;
    std::vector<double> f[5];
    for (int k = 0; k < 5; ++k) f[k].assign(n, 0.0);
    for (int z = 0; z < n; ++z) {
      const double T = z < n / 2 ? 1.0 : 0.7;
      f[0][z] = T * T * T;
      f[1][z] = 3.0 * T * T * T * T;
    }
    OK(rlb_batch_init(b, j, f[0].data(), f[1].data(), f[2].data(), f[3].data(), f[4].data(), 0));
  }
  const int64_t steps[3] = {10, 3, 7};
  OK(rlb_batch_step(b, steps));
  for (int j = 0; j < 3; ++j) {
    const int n = tubes[j].n;
    std::vector<double> nn(n), eps(n), U(4 * n), P(n);
    OK(rlb_batch_read(b, j, nn.data(), eps.data(), U.data(), P.data(), 0));
    uint32_t flags;
    int64_t t;
    OK(rlb_batch_status(b, j, &flags, &t));
    EXPECT(t == steps[j]);
  }
  rlb_batch_destroy(b);
  (void)hipFree(d);
  printf("batch order %d precision %d ok\n", order, precision);
  return 0;
}

static int server() {
  const size_t pool = size_t(1) << 30;
  void *d = nullptr;
  if (hipMalloc(&d, pool) != hipSuccess) return 1;
  rlb_server *sv = nullptr;
  OK(rlb_server_create(&sv, d, pool, 8, 8));
  std::vector<std::vector<double>> keep;
  std::vector<std::vector<double>> outs;
  int64_t ids[6];
  for (int r = 0; r < 6; ++r) {
    const bool tube = r % 3 != 2;
    const int nx = tube ? 1 : 16, ny = tube ? 1 : 12, nz = tube ? 300 + 50 * r : 10;
    std::vector<double> f[5];
    fields(nx, ny, nz, f);
    for (int k = 0; k < 5; ++k) keep.push_back(f[k]);
    const size_t C = (size_t)nx * ny * nz;
    outs.emplace_back(7 * C);
    double *o = outs.back().data();
    rlb_request q{};
    q.kind = tube ? RLB_REQ_TUBE : RLB_REQ_BOX;
    q.nx = nx; q.ny = ny; q.nz = nz;
    q.precision = r % 2 ? RLB_MIXED : RLB_FP64;
    q.tau_mode = RLB_TAU_ETA_S;
    q.order = r % 4 == 3 ? RLB_ORDER2 : RLB_ORDER3;
    q.eta_s = 0.1;
    q.steps = 20 + 3 * r;
    const size_t base = keep.size() - 5;
    q.n = keep[base].data(); q.eps = keep[base + 1].data(); q.vx = keep[base + 2].data();
    q.vy = keep[base + 3].data(); q.vz = keep[base + 4].data();
    q.out_n = o; q.out_eps = o + C; q.out_U4 = o + 2 * C; q.out_P = o + 6 * C;
    EXPECT(rlb_request_bytes(&q) > 0);
    OK(rlb_server_submit(sv, &q, &ids[r]));
  }
  int done = 0;
  for (int it = 0; it < 600 && done < 6; ++it) {
    rlb_completion c[8];
    int32_t cnt = 0;
    OK(rlb_server_poll(sv, c, 8, &cnt, 100));
    for (int i = 0; i < cnt; ++i) EXPECT(c[i].rc == RLB_OK);
    done += cnt;
  }
  EXPECT(done == 6);
  int64_t pending, rounds;
  OK(rlb_server_pending(sv, &pending, &rounds));
  EXPECT(pending == 0);
  rlb_server_destroy(sv);
  (void)hipFree(d);
  printf("server ok (%lld rounds)\n", (long long)rounds);
  return 0;
}

static int run();
// stdout unbuffered; leave with _exit so that the runtime's own teardown
// (outside this test) does not run under the sanitizer allocator
int main() {
  setvbuf(stdout, nullptr, _IONBF, 0);
  const int rc = run();
  printf(rc ? "FAILED\n" : "all ok\n");
  _exit(rc);
}

static int run() {
  rlb_lattice_t lat;
  OK(rlb_lattice_info(3, &lat));
  OK(rlb_lattice_info(2, &lat));
  EXPECT(rlb_lattice_info(5, &lat) == RLB_EINVAL);
  EXPECT(rlb_state_bytes(0, 4, 4, RLB_FP64, 3, 0) == 0);
  EXPECT(rlb_strerror(-99) != nullptr);
  rlb_solver *bad = nullptr;
  rlb_config cfg{8, 8, 8, RLB_FP64, RLB_TAU_FIXED, 0.4, 0.0, 3, 0};
  EXPECT(rlb_create(&bad, &cfg, (void *)(uintptr_t)4096, 1 << 30, nullptr) == RLB_EINVAL);
  for (int order : {3, 2})
    for (int prec : {RLB_FP64, RLB_MIXED}) {
      if (box(order, prec, RLB_PATTERN_AB, false)) return 1;
      if (box(order, prec, RLB_PATTERN_AA, false)) return 1;
      if (box(order, prec, RLB_PATTERN_AB, true)) return 1;
      if (batch(order, prec)) return 1;
    }
  if (server()) return 1;
  return 0;
}
