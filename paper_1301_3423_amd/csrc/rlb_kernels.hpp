// Kernels of one periodic box.  One thread owns one cell; a block of 256
// threads covers 256 consecutive cells in x-fastest order.
//
// Storage (per population i, x fastest, `stride` elements apart):
//   the current buffer holds, for the current time t, values that land on
//   cell x when streamed:  cur[i][x - theta_i] = f_i(x, t).
// So gathering cur[i][x - theta_i] yields the pre-collision state f(x, t)
// (pull streaming, Eq. rlb:disc left side), and a step writes the
// post-collision values of cell x to nxt[i][x], which is again of that
// form for time t + 1.
#pragma once

#include "rlb_device.hpp"

namespace rlb {

inline constexpr int BLOCK = 256;

template <class S>
__device__ __forceinline__ S load_at(const S *base, int cell) {
  const uint32_t boff = static_cast<uint32_t>(cell) * static_cast<uint32_t>(sizeof(S));
  return *reinterpret_cast<const S *>(reinterpret_cast<const char *>(base) + boff);
}

template <class S>
__device__ __forceinline__ void store_at(S *base, int cell, S v) {
  const uint32_t boff = static_cast<uint32_t>(cell) * static_cast<uint32_t>(sizeof(S));
  *reinterpret_cast<S *>(reinterpret_cast<char *>(base) + boff) = v;
}

__device__ __forceinline__ void cell_coords(int cell, const Geom &g, int &x, int &y, int &z) {
  x = cell % g.nx;
  const int yz = cell / g.nx;
  y = yz % g.ny;
  z = yz / g.ny;
}

// Gather f_i(x, t) for all 128 points (pull streaming).
template <class S>
__device__ __forceinline__ void gather(const S *__restrict__ cur, const Geom &g, const Shifts &sh,
                                       S (&f)[Q]) {
  static_for<0, Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr Point P = D3Q128[i];
    f[i] = load_at(cur + i * g.stride, sh.back<P.tx, P.ty, P.tz>());
  });
}

// Equilibrium (Eq. disc1) and Anderson-Witting relaxation (Eq. rlb:disc
// right side) of all points of one cell, written through `put(i, value)`.
// The rate p_i^mu U_mu / (tau p_i^0) = (gamma/tau)(1 - theta_i.v/R)
// = g - t_i for point i and g + t_i for its inverse.
template <class S, class Put>
__device__ __forceinline__ void relax_cell(const S (&f)[Q], const Frame &fr, double tau, Put &&put) {
  using CT = S; // per-population arithmetic in the storage precision
  const EqCoef e = eq_coefficients(fr.n, fr.T, fr.U0, fr.Ux, fr.Uy, fr.Uz);
  const double g = fr.U0 / tau;
  const CT gg = CT(g);
  const CT bx = CT(g * fr.vx * INV_R), by = CT(g * fr.vy * INV_R), bz = CT(g * fr.vz * INV_R);
  static_for<0, NSHELL>([&](auto L) {
    constexpr int l = decltype(L)::value;
    const ShellCoef<CT> s = shell_coefficients<l, CT>(e);
    static_for<shell_pair_begin(l), shell_pair_begin(l + 1)>([&](auto K) {
      constexpr int k = decltype(K)::value;
      constexpr Point P = D3Q128[2 * k];
      CT E, O;
      shell_eval<2 * k, CT>(s, E, O);
      const CT wE = CT(P.w) * E, wO = CT(P.w) * O;
      CT t = CT(0);
      if constexpr (P.tx != 0) t = fmadd(CT(P.tx), bx, t);
      if constexpr (P.ty != 0) t = fmadd(CT(P.ty), by, t);
      if constexpr (P.tz != 0) t = fmadd(CT(P.tz), bz, t);
      const CT a = f[2 * k], b = f[2 * k + 1];
      const CT fa = fmadd(gg - t, (wE + wO) - a, a);
      const CT fb = fmadd(gg + t, (wE - wO) - b, b);
      put(std::integral_constant<int, 2 * k>{}, fa);
      put(std::integral_constant<int, 2 * k + 1>{}, fb);
    });
  });
}

// One time step: gather, moments, Landau frame, tau, equilibrium,
// relaxation, aligned store of the post-collision values.
template <class S>
__global__ void __launch_bounds__(BLOCK) k_step(const S *__restrict__ cur, S *__restrict__ nxt, Geom g,
                                                Relax rx, unsigned *__restrict__ status) {
  const int cell = blockIdx.x * BLOCK + threadIdx.x;
  if (cell >= g.cells) return;
  int x, y, z;
  cell_coords(cell, g, x, y, z);
  const Shifts sh(x, y, z, g);
  S f[Q];
  gather(cur, g, sh, f);
  const Moments m = moments(f);
  Frame fr;
  unsigned flags = landau_frame(m, fr);
  const double tau = relaxation_time(rx, fr.n, fr.T);
  relax_cell(f, fr, tau, [&](auto I, S v) {
    constexpr int i = decltype(I)::value;
    store_at(nxt + i * g.stride, cell, v);
  });
  if (flags) atomicOr(status, flags);
}

// Initial state: local equilibrium of (n, eps, v) in every cell, stored so
// that the next gather returns it (scatter to x - theta_i).
template <class S>
__global__ void __launch_bounds__(BLOCK) k_init(const double *__restrict__ n_, const double *__restrict__ eps_,
                                                const double *__restrict__ vx_, const double *__restrict__ vy_,
                                                const double *__restrict__ vz_, S *__restrict__ cur, Geom g,
                                                unsigned *__restrict__ status) {
  const int cell = blockIdx.x * BLOCK + threadIdx.x;
  if (cell >= g.cells) return;
  int x, y, z;
  cell_coords(cell, g, x, y, z);
  const Shifts sh(x, y, z, g);
  const double n = n_[cell], eps = eps_[cell], vx = vx_[cell], vy = vy_[cell], vz = vz_[cell];
  const double v2 = vx * vx + vy * vy + vz * vz;
  unsigned flags = 0;
  if (!(n > 0.0) || !(eps > 0.0) || !(v2 < 1.0)) flags |= FLAG_NONPHYSICAL;
  if (!__builtin_isfinite(n + eps + v2)) flags |= FLAG_NONFINITE;
  const double gamma = 1.0 / __builtin_sqrt(1.0 - v2);
  const double T = eps / (3.0 * n);
  const EqCoef e = eq_coefficients(n, T, gamma, gamma * vx, gamma * vy, gamma * vz);
  using CT = double;
  static_for<0, NSHELL>([&](auto L) {
    constexpr int l = decltype(L)::value;
    const ShellCoef<CT> s = shell_coefficients<l, CT>(e);
    static_for<shell_pair_begin(l), shell_pair_begin(l + 1)>([&](auto K) {
      constexpr int k = decltype(K)::value;
      constexpr Point P = D3Q128[2 * k];
      CT E, O;
      shell_eval<2 * k, CT>(s, E, O);
      store_at(cur + (2 * k) * g.stride, sh.back<P.tx, P.ty, P.tz>(), S(P.w * (E + O)));
      store_at(cur + (2 * k + 1) * g.stride, sh.back<-P.tx, -P.ty, -P.tz>(), S(P.w * (E - O)));
    });
  });
  if (flags) atomicOr(status, flags);
}

// Macroscopic fields of the current pre-collision state.
template <class S>
__global__ void __launch_bounds__(BLOCK) k_read(const S *__restrict__ cur, Geom g, double *__restrict__ n_,
                                                double *__restrict__ eps_, double *__restrict__ U_,
                                                double *__restrict__ P_, unsigned *__restrict__ status) {
  const int cell = blockIdx.x * BLOCK + threadIdx.x;
  if (cell >= g.cells) return;
  int x, y, z;
  cell_coords(cell, g, x, y, z);
  const Shifts sh(x, y, z, g);
  S f[Q];
  gather(cur, g, sh, f);
  const Moments m = moments(f);
  Frame fr;
  const unsigned flags = landau_frame(m, fr);
  if (n_) n_[cell] = fr.n;
  if (eps_) eps_[cell] = fr.eps;
  if (P_) P_[cell] = fr.eps / 3.0;
  if (U_) {
    U_[cell] = fr.U0;
    U_[g.cells + cell] = fr.Ux;
    U_[2 * g.cells + cell] = fr.Uy;
    U_[3 * g.cells + cell] = fr.Uz;
  }
  if (flags) atomicOr(status, flags);
}

// Per-population sums over all cells (streaming keeps each of them), in a
// fixed order: pass 1 writes one partial per (population, block) with a
// tree reduction over the block; pass 2 reduces the partials of each
// population the same way.
inline constexpr int SUM_CELLS_PER_THREAD = 16;

template <class S>
__global__ void __launch_bounds__(BLOCK) k_popsum_partial(const S *__restrict__ cur, Geom g,
                                                          double *__restrict__ partial, int nblocks) {
  __shared__ double red[BLOCK];
  const int i = blockIdx.y;
  const S *base = cur + i * g.stride;
  const int chunk = BLOCK * SUM_CELLS_PER_THREAD;
  const int c0 = blockIdx.x * chunk;
  double acc = 0.0;
  for (int j = 0; j < SUM_CELLS_PER_THREAD; ++j) {
    const int c = c0 + j * BLOCK + threadIdx.x;
    if (c < g.cells) acc += static_cast<double>(base[c]);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = BLOCK / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[i * nblocks + blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(BLOCK) k_popsum_final(const double *__restrict__ partial, int nblocks,
                                                        double *__restrict__ total) {
  __shared__ double red[BLOCK];
  const int i = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += BLOCK) acc += partial[i * nblocks + b];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = BLOCK / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) total[i] = red[0];
}

} // namespace rlb
