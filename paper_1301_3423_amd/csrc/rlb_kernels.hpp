// Kernels of one periodic box.  Cells are numbered x fastest; population i
// of cell c lives at the tiled element (c / TILE) * Q * TILE + i * TILE +
// c % TILE of a buffer (see tile_elem), written cur[i][c] below.
//
// Storage: the current buffer holds, for the current time t, values that
//   land on cell x when streamed:  cur[i][x - theta_i] = f_i(x, t).
// So gathering cur[i][x - theta_i] yields the pre-collision state f(x, t)
// (pull streaming, Eq. rlb:disc left side), and a step writes the
// post-collision values of cell x to nxt[i][x], which is again of that
// form for time t + 1.
#pragma once

#include "rlb_device.hpp"

namespace rlb {

inline constexpr int BLOCK = 256;

// How a step reads and writes its populations (slot (i, x) = population i
// of cell x in a buffer):
//   PULL     two buffers: gather cur[i][x - theta_i], store nxt[i][x];
//   AA_EVEN  one buffer in its natural state, slot (i, x) = f_i(x): read
//            slot (i, x), store the post-collision f_i to slot (inv(i), x);
//   AA_ODD   one buffer in the swapped state, slot (inv(i), x - theta_i) =
//            f_i(x): read those slots and store the post-collision f_i to
//            slot (i, x + theta_i), which is the natural state again.
// An AA step writes exactly the slots its own cell read, so the update is
// in place (the "AA" streaming pattern): one buffer instead of two.
// AA_ODD_WIDE is AA_ODD for boxes with nx > MAXD, where the two-lane kernel
// computes the wrapped x of each store on the spot instead of keeping a
// table of them live (which made the float64 kernel spill).
// AA_ODD_ROT is AA_ODD for the one-lane row kernel when every block holds
// whole rows (nx divides the block size): the post-collision values are
// first rotated along x through LDS, so that every wavefront stores whole,
// aligned 256-byte segments instead of segments shifted by theta_x.
enum Access { PULL = 0, AA_EVEN = 1, AA_ODD = 2, AA_ODD_WIDE = 3, AA_ODD_ROT = 4 };

constexpr bool aa_odd(int ac) { return ac == AA_ODD || ac == AA_ODD_WIDE || ac == AA_ODD_ROT; }

// (c + s) mod n for |s| <= MAXD < n.  Below zero c + s wraps to a huge
// unsigned value, which min(t, t + n) replaces by t + n; at or above n,
// min(t, t - n) picks t - n (t - n wraps to a huge value when t < n).
__device__ __forceinline__ int wrap_fwd_wide(int c, int s, int n) {
  unsigned t = static_cast<unsigned>(c + s);
  const unsigned nu = static_cast<unsigned>(n);
  const unsigned up = t + nu;
  t = up < t ? up : t;
  const unsigned dn = t - nu;
  t = dn < t ? dn : t;
  return static_cast<int>(t);
}

// Population pointers of a step: restrict-qualified for the two-buffer
// pull, plain for the in-place AA steps (there cur == nxt).
template <class S, int AC>
using InPtr = std::conditional_t<AC == PULL, const S *__restrict__, const S *>;
template <class S, int AC>
using OutPtr = std::conditional_t<AC == PULL, S *__restrict__, S *>;

template <class S>
__device__ __forceinline__ S load_at(const S *base, int cell) {
  const uint32_t boff = static_cast<uint32_t>(cell) * static_cast<uint32_t>(sizeof(S));
  return *reinterpret_cast<const S *>(reinterpret_cast<const char *>(base) + boff);
}

// Post-collision values are not read again before the whole lattice has
// streamed through the caches, so they are stored non-temporally (measured
// +2-3 % on the step kernels; non-temporal loads were slower).
template <class S>
__device__ __forceinline__ void store_at(S *base, int cell, S v) {
  const uint32_t boff = static_cast<uint32_t>(cell) * static_cast<uint32_t>(sizeof(S));
  __builtin_nontemporal_store(v, reinterpret_cast<S *>(reinterpret_cast<char *>(base) + boff));
}

// Ordinary store, for the odd AA step: its stores land at x + theta_i, so a
// wavefront's 64 values straddle cache lines that neighbouring wavefronts
// complete; through the cache those partial lines merge before they reach
// HBM (measured at 256^3: the odd step 11 % faster in float32 and 8 % in
// float64 than with non-temporal stores).
template <class S>
__device__ __forceinline__ void store_plain(S *base, int cell, S v) {
  const uint32_t boff = static_cast<uint32_t>(cell) * static_cast<uint32_t>(sizeof(S));
  *reinterpret_cast<S *>(reinterpret_cast<char *>(base) + boff) = v;
}

// Loads and stores at a 64-bit element index (tiled storage of boxes of
// any size); the plain store is for the odd AA step, as store_plain.
template <class S>
__device__ __forceinline__ S load_e(const S *base, int64_t e) {
  return base[e];
}
template <class S>
__device__ __forceinline__ void store_e(S *base, int64_t e, S v) {
  __builtin_nontemporal_store(v, base + e);
}
template <class S>
__device__ __forceinline__ void store_e_plain(S *base, int64_t e, S v) {
  base[e] = v;
}

__device__ __forceinline__ void cell_coords(int cell, const Geom &g, int &x, int &y, int &z) {
  x = cell % g.nx;
  const int yz = cell / g.nx;
  y = yz % g.ny;
  z = yz / g.ny;
}

// Gather f_i(x, t) for all points of the model from a buffer laid out for
// `mode` (an Access value: PULL storage, or the natural or swapped AA state).
template <class M, class S>
__device__ __forceinline__ void gather(const S *__restrict__ cur, const Geom &g, const Shifts &sh,
                                       S (&f)[M::Q], int mode = PULL, int cell = 0) {
  constexpr int T = TILE<S>;
  static_for<0, M::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr Point P = M::P[i];
    if (mode == AA_EVEN)
      f[i] = load_e(cur + i * T, tile_elem<M, S>(cell));
    else if (mode == AA_ODD)
      f[i] = load_e(cur + (i ^ 1) * T, tile_elem<M, S>(sh.back<P.tx, P.ty, P.tz>()));
    else
      f[i] = load_e(cur + i * T, tile_elem<M, S>(sh.back<P.tx, P.ty, P.tz>()));
  });
}

// Equilibrium (Eq. disc1) and Anderson-Witting relaxation (Eq. rlb:disc
// right side) of all points of one cell: pre-collision values come from
// `get(i)`, post-collision values go out through `put(i, value)`.
// The rate p_i^mu U_mu / (tau p_i^0) = (gamma/tau)(1 - theta_i.v/R)
// = g - t_i for point i and g + t_i for its inverse.
template <class M, class S, class Get, class Put>
__device__ __forceinline__ void relax_cell(Get &&get, const Frame &fr, double tau, Put &&put) {
  using CT = S; // per-population arithmetic in the storage precision
  const EqCoef<M> e = eq_coefficients<M>(fr.n, fr.T, fr.U0, fr.Ux, fr.Uy, fr.Uz);
  const double g = fr.U0 / tau;
  const CT gg = CT(g);
  const CT bx = CT(g * fr.vx * M::INV_R), by = CT(g * fr.vy * M::INV_R), bz = CT(g * fr.vz * M::INV_R);
  static_for<0, M::NSHELL>([&](auto L) {
    constexpr int l = decltype(L)::value;
    const ShellCoef<M, CT> s = shell_coefficients<M, l, CT>(e);
    static_for<shell_pair_begin<M>(l), shell_pair_begin<M>(l + 1)>([&](auto K) {
      constexpr int k = decltype(K)::value;
      constexpr Point P = M::P[2 * k];
      CT E, O;
      shell_eval<M, 2 * k, CT>(s, E, O);
      const CT wE = CT(P.w) * E, wO = CT(P.w) * O;
      CT t = CT(0);
      if constexpr (P.tx != 0) t = fmadd(CT(P.tx), bx, t);
      if constexpr (P.ty != 0) t = fmadd(CT(P.ty), by, t);
      if constexpr (P.tz != 0) t = fmadd(CT(P.tz), bz, t);
      const CT a = get(std::integral_constant<int, 2 * k>{}), b = get(std::integral_constant<int, 2 * k + 1>{});
      const CT fa = fmadd(gg - t, (wE + wO) - a, a);
      const CT fb = fmadd(gg + t, (wE - wO) - b, b);
      put(std::integral_constant<int, 2 * k>{}, fa);
      put(std::integral_constant<int, 2 * k + 1>{}, fb);
    });
  });
}

// ---- the time step: one cell on two lanes ---------------------------------
//
// Lanes c and c + 32 of a wavefront share cell c of the wave's 32 cells:
// the lane with member m = 0 holds point 2k of every inversion pair k, the
// lane with m = 1 holds point 2k + 1, whose displacement, odd monomials and
// relaxation asymmetry are those of point 2k with the sign
// sigma = 1 - 2m.  Each lane therefore runs the same instruction stream
// with the same immediates: sigma enters once, in the gather offsets, the
// odd moments, the odd equilibrium coefficients and the velocity.  The 14
// moments are summed across the two lanes (identical results in both), and
// both lanes solve the same Landau problem.
// Block sizes of the step kernels, for access AC.  Small blocks run in
// different phases on one CU, so one block's arithmetic overlaps another's
// loads: the pull steps use 128 threads (tiled storage, 256^3: float64
// 6.24 ms against 6.31 ms with 64 threads, 6.44 ms with 256 and 6.75 ms with
// 512; mixed 3.06 ms against 3.15 ms with 256).  The AA steps, whose even
// step reads and writes only its own tiles, run best in 256-thread blocks
// (even step 2.87 ms mixed and 5.86 ms float64 against 3.05 and 6.04 ms with
// 64 threads).  The third-order float64 stash takes 256 B per thread.
template <int AC>
inline constexpr int step_block = AC == PULL ? 128 : 256;
template <class M, class S, int AC = PULL>
inline constexpr int pair_block = step_block<AC>;

// (c - s) mod n for a shift s known only at run time, |s| <= MAXD.
__device__ __forceinline__ int wrap_rt(int c, int s, int n) {
  if (n > MAXD) {
    int t = c - s;
    t += (t < 0) ? n : 0;
    t -= (t >= n) ? n : 0;
    return t;
  }
  if (n == 1) return 0;
  return (c - s + (MAXD + 1) * n) % n;
}

// Per-lane gather offsets of the member with sign sigma: the source cell
// x - sigma*s along each axis, as cell-index parts.
struct HalfShifts {
  int xo[2 * MAXD + 1], yo[2 * MAXD + 1], zo[2 * MAXD + 1];
  __device__ __forceinline__ HalfShifts(int x, int y, int z, int sigma, const Geom &g) {
#pragma unroll
    for (int s = -MAXD; s <= MAXD; ++s) {
      xo[s + MAXD] = wrap_rt(x, sigma * s, g.nx);
      yo[s + MAXD] = wrap_rt(y, sigma * s, g.ny) * g.nx;
      zo[s + MAXD] = wrap_rt(z, sigma * s, g.nz) * (g.nx * g.ny);
    }
  }
  template <int TX, int TY, int TZ>
  __device__ __forceinline__ int back() const {
    return zo[TZ + MAXD] + yo[TY + MAXD] + xo[TX + MAXD];
  }
};

__device__ __forceinline__ double add_partner(double v) { return v + __shfl_xor(v, 32); }


// Float64 populations of the last stash_n pairs of the third-order model
// wait in LDS between the moment sums and the relaxation (256 B per thread:
// 64 KB per 256-thread step block, 128 KB per 512-thread tube workgroup),
// which keeps the live registers of the
// float64 kernels within two waves per SIMD.  The 33 pairs of the second-order model fit
// in registers.
template <class M, class S, int AC = PULL>
inline constexpr int stash_n = (sizeof(S) == 8 && M::Q == 128) ? 32 : 0;
template <class M, class S, int AC = PULL>
inline constexpr int stash_begin = M::Q / 2 - stash_n<M, S, AC>;
// LDS rows to declare (at least one)
template <class M, class S, int AC = PULL>
inline constexpr int stash_rows = stash_n<M, S, AC> > 0 ? stash_n<M, S, AC> : 1;

// One lattice update of `cell` by the two lanes (c, c + 32) of a wavefront
// (see above); `lds` is the block's stash of the last shell (float64 only,
// [stash_n][block size]).  Cells at or beyond g.cells are computed for a
// clamped cell and never stored; with WALLS, solid cells (solid[cell] != 0)
// are computed but never stored either.  OR-s this cell's flags into `flags`.
// AC selects the access (PULL, AA_EVEN, AA_ODD, AA_ODD_WIDE); for AA,
// cur == nxt.
template <class M, class S, int TB, bool WALLS = false, int AC = PULL>
__device__ __forceinline__ void pair_cell_step(InPtr<S, AC> cur, OutPtr<S, AC> nxt, const Geom &g,
                                               const Relax &rx, int cell, S (*lds)[TB], unsigned &flags,
                                               const uint8_t *__restrict__ solid = nullptr) {
  constexpr int NPAIR = M::Q / 2;
  constexpr int STASH_BEGIN = stash_begin<M, S, AC>;
  const int lane = threadIdx.x & 63;
  const int m = lane >> 5;
  const int sigma = 1 - 2 * m;
  bool active = cell < g.cells;
  if (!active) cell = g.cells - 1; // keeps the partner exchange whole; never stored
  if constexpr (WALLS) active = active && solid[cell] == 0;
  int x, y, z;
  cell_coords(cell, g, x, y, z);
  constexpr int T = TILE<S>;
  S f[NPAIR];
  if constexpr (AC == AA_EVEN) {
    // own slot (2k + m, x)
    const int64_t own = tile_elem<M, S>(cell) + m * T;
    static_for<0, NPAIR>([&](auto K) {
      constexpr int k = decltype(K)::value;
      f[k] = load_e(cur + (2 * k) * T, own);
    });
  } else {
    // PULL: slot (2k + m, x - sigma theta); AA_ODD: slot (2k + 1 - m, x - sigma theta)
    const HalfShifts sh(x, y, z, sigma, g);
    const int mT = (aa_odd(AC) ? 1 - m : m) * T;
    static_for<0, NPAIR>([&](auto K) {
      constexpr int k = decltype(K)::value;
      constexpr Point P = M::P[2 * k];
      f[k] = load_e(cur + (2 * k) * T, tile_elem<M, S>(sh.back<P.tx, P.ty, P.tz>()) + mT);
    });
  }
  // moments of this lane's members; odd sums carry theta of point 2k
  Moments mo{};
  static_for<0, M::NSHELL>([&](auto L) {
    constexpr int l = decltype(L)::value;
    ShellSums a{};
    static_for<shell_pair_begin<M>(l), shell_pair_begin<M>(l + 1)>([&](auto K) {
      constexpr int k = decltype(K)::value;
      const double v = static_cast<double>(f[k]);
      a.template add_pair<M, k>(v, v);
    });
    a.template fold<M, l>(mo);
  });
  constexpr bool stash = stash_n<M, S, AC> > 0;
  if constexpr (stash) {
    static_for<STASH_BEGIN, NPAIR>([&](auto K) {
      constexpr int k = decltype(K)::value;
      lds[k - STASH_BEGIN][threadIdx.x] = f[k];
    });
    // compiler-only fence: the values must really be reloaded from LDS
    // later (forwarding the stores would keep them in registers)
    asm volatile("" ::: "memory");
  }
  const double sg = static_cast<double>(sigma);
  mo.Nx *= sg;
  mo.Ny *= sg;
  mo.Nz *= sg;
  mo.T0x *= sg;
  mo.T0y *= sg;
  mo.T0z *= sg;
  mo.N0 = add_partner(mo.N0);
  mo.Nx = add_partner(mo.Nx);
  mo.Ny = add_partner(mo.Ny);
  mo.Nz = add_partner(mo.Nz);
  mo.T00 = add_partner(mo.T00);
  mo.T0x = add_partner(mo.T0x);
  mo.T0y = add_partner(mo.T0y);
  mo.T0z = add_partner(mo.T0z);
  mo.Txx = add_partner(mo.Txx);
  mo.Tyy = add_partner(mo.Tyy);
  mo.Tzz = add_partner(mo.Tzz);
  mo.Txy = add_partner(mo.Txy);
  mo.Txz = add_partner(mo.Txz);
  mo.Tyz = add_partner(mo.Tyz);
  Frame fr;
  const unsigned fl = landau_frame(mo, fr);
  const double tau = relaxation_time<M>(rx, fr.n, fr.T);
  EqCoef<M> e = eq_coefficients<M>(fr.n, fr.T, fr.U0, fr.Ux, fr.Uy, fr.Uz);
  // coefficients of spatially odd monomials change sign for the inverse member
  static_for<0, M::NM>([&](auto A) {
    constexpr int j = decltype(A)::value;
    constexpr Mono mo_j = M::MONO[j];
    if constexpr ((mo_j.ax + mo_j.ay + mo_j.az) % 2 != 0) e.c[j] *= sg;
  });
  using CT = S;
  const double gdt = fr.U0 / tau;
  const CT gg = CT(gdt);
  const double gs = gdt * M::INV_R * sg;
  const CT bx = CT(gs * fr.vx), by = CT(gs * fr.vy), bz = CT(gs * fr.vz);
  // AA_ODD stores go to x + sigma theta: the offsets of x - (-sigma) theta;
  // AA_ODD_WIDE keeps only the y and z parts and wraps x per store
  struct NoShifts {
    __device__ NoShifts(int, int, int, int, const Geom &) {}
  };
  struct YZShifts {
    int yo[2 * MAXD + 1], zo[2 * MAXD + 1];
    __device__ __forceinline__ YZShifts(int, int y, int z, int sigma, const Geom &g) {
#pragma unroll
      for (int s = -MAXD; s <= MAXD; ++s) {
        yo[s + MAXD] = wrap_rt(y, sigma * s, g.ny) * g.nx;
        zo[s + MAXD] = wrap_rt(z, sigma * s, g.nz) * (g.nx * g.ny);
      }
    }
  };
  using Fwd = std::conditional_t<AC == AA_ODD, HalfShifts, std::conditional_t<AC == AA_ODD_WIDE, YZShifts, NoShifts>>;
  const Fwd fwd(x, y, z, -sigma, g);
  // PULL: slot (2k + m, x); AA_EVEN: slot (2k + 1 - m, x); AA_ODD: slot
  // (2k + m, x + sigma theta), whose offsets depend on the point
  const int64_t out_off = tile_elem<M, S>(cell) + (AC == AA_EVEN ? 1 - m : m) * T;
  static_for<0, M::NSHELL>([&](auto L) {
    constexpr int l = decltype(L)::value;
    const ShellCoef<M, CT> s = shell_coefficients<M, l, CT>(e);
    static_for<shell_pair_begin<M>(l), shell_pair_begin<M>(l + 1)>([&](auto K) {
      constexpr int k = decltype(K)::value;
      constexpr Point P = M::P[2 * k];
      CT E, O;
      shell_eval<M, 2 * k, CT>(s, E, O);
      const CT feq = CT(P.w) * (E + O);
      CT t = CT(0);
      if constexpr (P.tx != 0) t = fmadd(CT(P.tx), bx, t);
      if constexpr (P.ty != 0) t = fmadd(CT(P.ty), by, t);
      if constexpr (P.tz != 0) t = fmadd(CT(P.tz), bz, t);
      CT a;
      if constexpr (stash && k >= STASH_BEGIN)
        a = lds[k - STASH_BEGIN][threadIdx.x];
      else
        a = f[k];
      const CT fs = fmadd(gg - t, feq - a, a);
      if constexpr (AC == AA_ODD_WIDE) {
        // a fresh copy of x per store keeps the compiler from computing the
        // 13 wrapped values once and holding them through the arithmetic
        int xs = x;
        asm volatile("" : "+v"(xs));
        const int dst = fwd.zo[MAXD + P.tz] + fwd.yo[MAXD + P.ty] + wrap_fwd_wide(xs, sigma * P.tx, g.nx);
        if (active) store_e_plain(nxt + (2 * k) * T, tile_elem<M, S>(dst) + m * T, S(fs));
      } else if constexpr (AC == AA_ODD) {
        if (active)
          store_e_plain(nxt + (2 * k) * T, tile_elem<M, S>(fwd.template back<P.tx, P.ty, P.tz>()) + m * T, S(fs));
      } else {
        if (active) store_e(nxt + (2 * k) * T, out_off, S(fs));
      }
    });
  });
  if (active) flags |= fl;
}


// Block order of the step kernels: each XCD takes a contiguous eighth of
// the lattice.  The hardware deals workgroups round-robin to the 8 XCDs
// (physical block b runs on XCD b % 8), so block b works on block
// (b % 8) * nb / 8 + b / 8; the mapping is a bijection when the count is a
// multiple of 8, and the identity otherwise.  With the tiled storage the
// tiles an XCD reads and writes then lie together, and the shifted gathers
// of neighbouring blocks meet in one L2 (256^3: mixed step 3.11 ms instead
// of 3.17 ms in plain order, float64 6.46 instead of 6.64).
__device__ __forceinline__ int pair_block_order(int b, int nb) {
  if (nb % 8) return b;
  return (b & 7) * (nb >> 3) + (b >> 3);
}

template <class M, class S, bool WALLS, int AC = PULL>
__global__ void __launch_bounds__((pair_block<M, S, AC>)) __attribute__((amdgpu_waves_per_eu(2)))
k_step(InPtr<S, AC> cur, OutPtr<S, AC> nxt, Geom g, Relax rx, unsigned *__restrict__ status,
       const uint8_t *__restrict__ solid) {
  constexpr int TB = pair_block<M, S, AC>;
  __shared__ S lds[stash_rows<M, S, AC>][TB];
  const int blk = pair_block_order(blockIdx.x, gridDim.x);
  const int cell = blk * (TB / 2) + (threadIdx.x >> 6) * 32 + (threadIdx.x & 31);
  unsigned flags = 0;
  pair_cell_step<M, S, TB, WALLS, AC>(cur, nxt, g, rx, cell, lds, flags, solid);
  if (flags) atomicOr(status, flags);
}

// ---- many shock tubes in one persistent launch ----------------------------
//
// One workgroup per tube (taken from `order`, longest work first) runs all
// of that tube's steps.  Tubes are independent, so no workgroup ever waits
// on another, and every workgroup leaves after its own step count.
struct TubeDesc {
  int64_t off[2]; // element offsets of the tube's two population buffers
  int64_t steps;  // steps to take in this launch
  int32_t n;      // cells along z
  int32_t cur;    // buffer holding the current state
  int32_t mode;   // 0 fixed tau, 1 tau from eta/s
  int32_t spin_limit; // polls a wait may take before it gives up; 0: TUBE_SPIN_LIMIT
  double tau, eta_s;
};

inline constexpr int TUBE_BLOCK = 512; // one workgroup fills a CU at two waves per SIMD

// Inside a workgroup the tube is cut into chunks of one wavefront (64 cells
// in float32, one per lane; 32 in float64, two lanes per cell), and the
// work is the sequence of (step s, chunk c) in the order k = s * nch + c.
// Each wavefront takes the next k from a counter in LDS, waits until the
// chunks its gathers reach (c - 1, c and c + 1 in the interior -- a gather
// reaches at most 6 cells, less than a chunk -- see chunk_reach for the
// periodic wrap) have finished step s - 1, computes the chunk and marks it
// done.  Those chunks are the only ones that read the slots (c, s + 1)
// overwrites (they read them as input of step s - 1) and the only ones whose
// outputs (c, s) reads, so this is the whole dependence: there is no barrier
// between steps, a wavefront that finishes its chunk goes on with the next
// one, possibly of the next step, and neighbouring chunks are computed at
// nearly the same time, so the cache lines they share are fetched once.
// Every dependence of k is on smaller k, all of which were taken earlier,
// so the work always progresses.  A step count per chunk is kept modulo
// 256 (chunks in progress are at most a few steps apart).  Tubes with more
// chunks than the flag array holds take the barrier form (k_tubes_sync).
template <class S>
inline constexpr int TUBE_CHUNK = sizeof(S) == 8 ? 32 : 64;
// LDS flag bytes: float64 keeps 128 KB for its stash, float32 has no stash
template <class S>
inline constexpr int TUBE_FLOW_CHUNKS = sizeof(S) == 8 ? 24576 : 65536;
// polls of a wait before it gives up and flags the tube (about 0.2 s; a
// normal wait is a few microseconds); bounds every wait
inline constexpr int TUBE_SPIN_LIMIT = 1 << 22;
inline constexpr unsigned FLAG_TUBE_SYNC = 8u; // RLB_FLAG_STALL

__device__ __forceinline__ bool step_reached(const volatile uint8_t *done, int c, uint8_t s) {
  return static_cast<uint8_t>(done[c] - s) < 128u;
}

// The chunks whose cells the gathers of chunk c reach, cells
// [c * CH - MAXD, end + MAXD) taken modulo n: a cyclic run of chunks from
// `first`, `count` long.  Interior chunks need c - 1 .. c + 1; next to the
// periodic wrap a last chunk shorter than MAXD cells makes the run reach
// one chunk further; a tube shorter than that whole range needs every chunk.
// The relation is symmetric, so the same chunks are the only ones that read
// (as input of the previous step) the slots chunk c overwrites.
template <int CH>
__device__ __forceinline__ void chunk_reach(int c, int nch, int n, int &first, int &count) {
  const int start = c * CH, end = start + CH < n ? start + CH : n;
  if (end - start + 2 * MAXD >= n) {
    first = 0;
    count = nch;
    return;
  }
  int lo = start - MAXD; // here n > 2 * MAXD: one wrap at most
  if (lo < 0) lo += n;
  int hi = end - 1 + MAXD;
  if (hi >= n) hi -= n;
  first = lo / CH;
  // a run that wraps may come back into its first chunk
  count = hi >= lo ? hi / CH - first + 1 : nch - first + hi / CH + 1;
  if (count > nch) count = nch;
}

// One tube cell per lane (float32): the cell index is z, so each lane keeps
// the tiled offsets of its 13 wrapped z and every population base is
// wavefront-uniform (32-bit: a tube has at most 2^22 cells).
template <class M, class S>
__device__ __forceinline__ void tube_cell_step(const S *__restrict__ in, S *__restrict__ out, const Geom &g,
                                               const Relax &rx, int z, unsigned &flags) {
  constexpr int T = TILE<S>;
  const bool active = z < g.cells;
  const int zc = active ? z : g.cells - 1;
  int zo[2 * MAXD + 1];
#pragma unroll
  for (int s = -MAXD; s <= MAXD; ++s) zo[s + MAXD] = static_cast<int>(tile_elem<M, S>(wrap_back(zc, s, g.nz)));
  const int own = static_cast<int>(tile_elem<M, S>(zc));
  S f[M::Q];
  // loads at raised priority (512-tube batch in the earlier form with a
  // barrier per step: 4306 -> 4465 MLUPS; the same time either way now)
  __builtin_amdgcn_s_setprio(3);
  static_for<0, M::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr Point P = M::P[i];
    f[i] = load_at(in + i * T, zo[P.tz + MAXD]);
  });
  __builtin_amdgcn_sched_barrier(0);
  __builtin_amdgcn_s_setprio(0);
  const Moments m = moments<M>(f);
  Frame fr;
  const unsigned fl = landau_frame(m, fr);
  const double tau = relaxation_time<M>(rx, fr.n, fr.T);
  relax_cell<M, S>([&](auto I) { return f[decltype(I)::value]; }, fr, tau, [&](auto I, S v) {
    constexpr int i = decltype(I)::value;
    if (active) store_at(out + i * T, own, v);
  });
  if (active) flags |= fl;
}

// The tube's work in (step, chunk) order; `order` lists the workgroups'
// tubes, each with at most TUBE_FLOW_CHUNKS<S> chunks and fewer than 2^31
// (step, chunk) items in this launch (the host splits longer runs).
template <class M, class S>
__global__ void __launch_bounds__(TUBE_BLOCK) __attribute__((amdgpu_waves_per_eu(2)))
k_tubes(S *__restrict__ base, const TubeDesc *__restrict__ desc, const int *__restrict__ order,
        unsigned *__restrict__ status) {
  constexpr bool f64 = sizeof(S) == 8;
  constexpr int TB = TUBE_BLOCK;
  constexpr int CH = TUBE_CHUNK<S>;
  __shared__ S lds[stash_rows<M, S>][f64 ? TB : 1];
  __shared__ uint8_t done_[TUBE_FLOW_CHUNKS<S>];
  __shared__ unsigned next_;
  const int j = __builtin_amdgcn_readfirstlane(order[blockIdx.x]);
  const TubeDesc d = desc[j]; // uniform: scalar loads
  Geom g;
  g.nx = 1;
  g.ny = 1;
  g.nz = d.n;
  g.cells = d.n;
  Relax rx;
  rx.mode = d.mode;
  rx.tau = d.tau;
  rx.eta_s = d.eta_s;
  const int lane = static_cast<int>(threadIdx.x) & 63;
  // float64: cell (lane & 31) of the wavefront's 32 on two lanes; float32:
  // one cell per lane
  const int slot = f64 ? (lane & 31) : lane;
  unsigned flags = 0;
  const unsigned nch = static_cast<unsigned>((d.n + CH - 1) / CH);
  volatile uint8_t *done = done_;
  for (unsigned c = threadIdx.x; c < nch; c += TB) done[c] = 0;
  if (threadIdx.x == 0) next_ = 0;
  __syncthreads();
  const unsigned total = static_cast<unsigned>(d.steps) * nch;
  const int spin_limit = d.spin_limit > 0 ? d.spin_limit : TUBE_SPIN_LIMIT;
  for (;;) {
    unsigned k = 0;
    if (lane == 0) k = atomicAdd(&next_, 1u);
    k = __builtin_amdgcn_readfirstlane(k);
    if (k >= total) break;
    const unsigned st = k / nch;
    const unsigned c = k - st * nch;
    int first, count;
    chunk_reach<CH>(static_cast<int>(c), static_cast<int>(nch), d.n, first, count);
    const uint8_t need = static_cast<uint8_t>(st);
    int spins = 0;
    for (;;) {
      bool ready = true;
      for (int q = 0, cq = first; q < count; ++q, cq = cq + 1 == static_cast<int>(nch) ? 0 : cq + 1)
        ready = ready && step_reached(done, cq, need);
      if (ready) break;
      if (++spins >= spin_limit) {
        flags |= FLAG_TUBE_SYNC; // never expected: give up the wait, keep going, report
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    // the neighbours' stores of step st - 1 are visible from here on
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const int cur = (d.cur + static_cast<int>(st & 1u)) & 1;
    const S *in = base + (cur ? d.off[1] : d.off[0]);
    S *out = base + (cur ? d.off[0] : d.off[1]);
    if constexpr (f64)
      pair_cell_step<M, S, TB>(in, out, g, rx, static_cast<int>(c) * CH + slot, lds, flags);
    else
      tube_cell_step<M, S>(in, out, g, rx, static_cast<int>(c) * CH + slot, flags);
    // this chunk's stores complete before it is marked done
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if (lane == 0) done[c] = static_cast<uint8_t>(st + 1);
  }
  if (flags) atomicOr(status + j, flags);
}

// Tubes beyond TUBE_FLOW_CHUNKS<S> chunks (float64 above 786,432 cells):
// every step in passes of TB / 2 (float64) or TB (float32) cells, with a
// workgroup barrier after each step (the step's stores are visible to the
// next gathers: all wavefronts of a workgroup share one CU).
template <class M, class S>
__global__ void __launch_bounds__(TUBE_BLOCK) __attribute__((amdgpu_waves_per_eu(2)))
k_tubes_sync(S *__restrict__ base, const TubeDesc *__restrict__ desc, const int *__restrict__ order,
             unsigned *__restrict__ status) {
  constexpr bool f64 = sizeof(S) == 8;
  constexpr int TB = TUBE_BLOCK;
  __shared__ S lds[stash_rows<M, S>][f64 ? TB : 1];
  const int j = __builtin_amdgcn_readfirstlane(order[blockIdx.x]);
  const TubeDesc d = desc[j];
  Geom g;
  g.nx = 1;
  g.ny = 1;
  g.nz = d.n;
  g.cells = d.n;
  Relax rx;
  rx.mode = d.mode;
  rx.tau = d.tau;
  rx.eta_s = d.eta_s;
  constexpr int per_pass = f64 ? TB / 2 : TB;
  const int slot = f64 ? (static_cast<int>(threadIdx.x) >> 6) * 32 + (threadIdx.x & 31) : static_cast<int>(threadIdx.x);
  const int wave0 = f64 ? (static_cast<int>(threadIdx.x) >> 6) * 32 : (static_cast<int>(threadIdx.x) & ~63);
  unsigned flags = 0;
  int cur = d.cur;
  for (int64_t st = 0; st < d.steps; ++st) {
    const S *in = base + (cur ? d.off[1] : d.off[0]);
    S *out = base + (cur ? d.off[0] : d.off[1]);
    for (int c0 = 0; c0 < d.n; c0 += per_pass) {
      if (c0 + wave0 >= d.n) continue; // wavefronts wholly beyond the tube skip the pass
      if constexpr (f64)
        pair_cell_step<M, S, TB>(in, out, g, rx, c0 + slot, lds, flags);
      else
        tube_cell_step<M, S>(in, out, g, rx, c0 + slot, flags);
    }
    __syncthreads();
    cur ^= 1;
  }
  if (flags) atomicOr(status + j, flags);
}

// ---- the time step for rows of 64k cells: one cell per lane ---------------
//
// When nx is a multiple of 64 every wavefront covers 64 consecutive cells
// of one row, so the y and z parts of each displacement are the same for
// the whole wavefront: they go into the scalar base address of each
// population array, and the lanes only carry the 13 wrapped x offsets.
// A lane owns a whole cell and uses the inversion pairs directly
// (s = f_i + f_inv(i) for the even moments, d = f_i - f_inv(i) for the odd
// ones, and f^eq = w (E +- O) for the two members).  With WALLS, lanes of
// solid cells leave at once.
// The odd AA step of the third-order model also keeps the 13 store offsets
// of x + theta_i live through the relaxation; the last row_stash populations
// then wait in LDS (24 KB per block), which keeps the kernel free of spills.
template <class M, class S, int AC>
inline constexpr int row_stash = ((AC == AA_ODD || AC == AA_ODD_ROT) && M::Q == 128) ? 24 : 0;

// Populations per LDS round of the rotated odd AA step (two buffers of
// rot_batch x block floats, so one barrier per round): 8 rounds of 16 in
// the third-order model, 3 of 22 in the second-order one.
template <class M>
inline constexpr int rot_batch = M::Q == 128 ? 16 : 22;
static_assert(M3::Q % rot_batch<M3> == 0 && M2::Q % rot_batch<M2> == 0);

template <class M, class S, bool WALLS, int AC = PULL>
__global__ void __launch_bounds__(step_block<AC>) __attribute__((amdgpu_waves_per_eu(2)))
k_step_row(InPtr<S, AC> cur, OutPtr<S, AC> nxt, Geom g, Relax rx, unsigned *__restrict__ status,
           const uint8_t *__restrict__ solid) {
  constexpr int RB = step_block<AC>;
  const int blk = pair_block_order(blockIdx.x, gridDim.x);
  int cell = blk * RB + threadIdx.x;
  // the rotated odd step has workgroup barriers: wavefronts beyond the last
  // cell stay, work on a copy of the last row and store nothing
  const bool active = cell < g.cells;
  if constexpr (AC == AA_ODD_ROT) {
    if (!active) cell = g.cells - g.nx + (threadIdx.x & 63) % g.nx;
  } else {
    if (!active) return; // whole wavefronts only: cells is a multiple of 64
  }
  if constexpr (WALLS) {
    if (solid[cell]) return;
  }
  constexpr int T = TILE<S>;
  const int x = cell % g.nx;
  const int row = __builtin_amdgcn_readfirstlane(cell / g.nx);
  const int y = row % g.ny, z = row / g.ny;
  const int nxny = g.nx * g.ny;
  // rows start on tile boundaries (nx % 64 == 0): a row starting at cell r
  // starts at element r * Q, and the lanes only carry the tiled x parts
  int xo[2 * MAXD + 1];
  int yo[2 * MAXD + 1], zo[2 * MAXD + 1]; // wavefront-uniform cell indices of row starts
#pragma unroll
  for (int sft = -MAXD; sft <= MAXD; ++sft) {
    xo[sft + MAXD] = tile_elem_x<M, S>(wrap_back(x, sft, g.nx));
    yo[sft + MAXD] = wrap_back(y, sft, g.ny) * g.nx;
    zo[sft + MAXD] = wrap_back(z, sft, g.nz) * nxny;
  }
  const auto rowp = [&](int r) { return static_cast<int64_t>(r) * M::Q; };
  S f[M::Q];
  const int64_t own_row = rowp(row * g.nx);
  const int own = tile_elem_x<M, S>(x);
  // (loads at raised wave priority, which helped the untiled storage, made
  // the tiled step about 1 % slower)
  static_for<0, M::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr Point P = M::P[i];
    if constexpr (AC == AA_EVEN)
      f[i] = load_at(cur + (i * T + own_row), own);
    else
      f[i] = load_at(cur + ((aa_odd(AC) ? i ^ 1 : i) * T + rowp(yo[P.ty + MAXD] + zo[P.tz + MAXD])),
                     xo[P.tx + MAXD]);
  });
  // keep the phases apart: interleaving them raises the register peak
  __builtin_amdgcn_sched_barrier(0);
  const Moments m = moments<M>(f);
  __builtin_amdgcn_sched_barrier(0);
  constexpr int RS = row_stash<M, S, AC>;
  constexpr int RS0 = M::Q - RS;
  __shared__ S lds[RS > 0 ? RS : 1][RB];
  if constexpr (RS > 0) {
    static_for<RS0, M::Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      lds[i - RS0][threadIdx.x] = f[i];
    });
    // compiler-only fence: the stashed values must really come back from LDS
    asm volatile("" ::: "memory");
  }
  const auto get = [&](auto I) -> S {
    constexpr int i = decltype(I)::value;
    if constexpr (i >= RS0)
      return lds[i - RS0][threadIdx.x];
    else
      return f[i];
  };
  Frame fr;
  const unsigned flags = landau_frame(m, fr);
  const double tau = relaxation_time<M>(rx, fr.n, fr.T);
  __builtin_amdgcn_sched_barrier(0);
  if constexpr (AC == AA_ODD_ROT) {
    // stores to x + theta_i, rotated along the row through LDS: population i
    // of this cell goes to LDS position (row start + (x + theta_x) mod nx);
    // after the round's barrier each lane takes the value at its own
    // position, which belongs to its own x in row (y + theta_y, z + theta_z),
    // and stores it aligned.  Rows lie wholly in the block (RB % nx == 0).
    constexpr int NB = rot_batch<M>;
    __shared__ S stage[2][NB][RB];
    const int rstart = static_cast<int>(threadIdx.x) - x; // block position of the row's first cell
    int xs = x;
    asm volatile("" : "+v"(xs));
    int lp[2 * MAXD + 1]; // LDS position of x - sft
#pragma unroll
    for (int sft = -MAXD; sft <= MAXD; ++sft) lp[sft + MAXD] = rstart + wrap_back(xs, sft, g.nx);
    relax_cell<M, S>(get, fr, tau, [&](auto I, S v) {
      constexpr int i = decltype(I)::value;
      constexpr Point P = M::P[i];
      constexpr int buf = (i / NB) & 1;
      if (active) stage[buf][i % NB][lp[MAXD - P.tx]] = v;
      if constexpr (i % NB == NB - 1) {
        // one barrier per round: a buffer is written again two rounds
        // later, after every lane has passed the next round's barrier
        __syncthreads();
        static_for<0, NB>([&](auto J) {
          constexpr int j = decltype(J)::value;
          constexpr int q = i - (NB - 1) + j;
          constexpr Point PQ = M::P[q];
          const S w = stage[buf][j][threadIdx.x];
          if (active) store_at(nxt + (q * T + rowp(yo[MAXD - PQ.ty] + zo[MAXD - PQ.tz])), own, w);
        });
      }
    });
  } else if constexpr (AC == AA_ODD) {
    // stores to x + theta_i; the x offsets are computed again here rather
    // than kept live through the arithmetic
    int xs = x;
    asm volatile("" : "+v"(xs));
    int xf[2 * MAXD + 1];
#pragma unroll
    for (int sft = -MAXD; sft <= MAXD; ++sft) xf[sft + MAXD] = tile_elem_x<M, S>(wrap_back(xs, sft, g.nx));
    relax_cell<M, S>(get, fr, tau, [&](auto I, S v) {
      constexpr int i = decltype(I)::value;
      constexpr Point P = M::P[i];
      store_plain(nxt + (i * T + rowp(yo[MAXD - P.ty] + zo[MAXD - P.tz])), xf[MAXD - P.tx], v);
    });
  } else {
    relax_cell<M, S>(get, fr, tau, [&](auto I, S v) {
      constexpr int i = decltype(I)::value;
      store_at(nxt + ((AC == AA_EVEN ? i ^ 1 : i) * T + own_row), own, v);
    });
  }
  if (active && flags) atomicOr(status, flags);
}

// Initial state: local equilibrium of (n, eps, v) in every cell, stored so
// that the next gather returns it (scatter to x - theta_i).
// With aa != 0 the state is written in the natural AA layout (slot (i, x) =
// f_i(x)) instead of scattered for the pull.
template <class M, class S>
__global__ void __launch_bounds__(BLOCK) k_init(const double *__restrict__ n_, const double *__restrict__ eps_,
                                                const double *__restrict__ vx_, const double *__restrict__ vy_,
                                                const double *__restrict__ vz_, S *__restrict__ cur, Geom g,
                                                unsigned *__restrict__ status, int aa) {
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
  const EqCoef<M> e = eq_coefficients<M>(n, T, gamma, gamma * vx, gamma * vy, gamma * vz);
  using CT = double;
  static_for<0, M::NSHELL>([&](auto L) {
    constexpr int l = decltype(L)::value;
    const ShellCoef<M, CT> s = shell_coefficients<M, l, CT>(e);
    static_for<shell_pair_begin<M>(l), shell_pair_begin<M>(l + 1)>([&](auto K) {
      constexpr int k = decltype(K)::value;
      constexpr Point P = M::P[2 * k];
      CT E, O;
      shell_eval<M, 2 * k, CT>(s, E, O);
      constexpr int T = TILE<S>;
      if (aa) {
        store_e(cur + (2 * k) * T, tile_elem<M, S>(cell), S(P.w * (E + O)));
        store_e(cur + (2 * k + 1) * T, tile_elem<M, S>(cell), S(P.w * (E - O)));
      } else {
        store_e(cur + (2 * k) * T, tile_elem<M, S>(sh.back<P.tx, P.ty, P.tz>()), S(P.w * (E + O)));
        store_e(cur + (2 * k + 1) * T, tile_elem<M, S>(sh.back<-P.tx, -P.ty, -P.tz>()), S(P.w * (E - O)));
      }
    });
  });
  if (flags) atomicOr(status, flags);
}

// Macroscopic fields of the current pre-collision state (zero at solid
// cells when `solid` is given).
template <class M, class S>
__global__ void __launch_bounds__(BLOCK) k_read(const S *__restrict__ cur, Geom g, double *__restrict__ n_,
                                                double *__restrict__ eps_, double *__restrict__ U_,
                                                double *__restrict__ P_, unsigned *__restrict__ status,
                                                const uint8_t *__restrict__ solid, int mode) {
  const int cell = blockIdx.x * BLOCK + threadIdx.x;
  if (cell >= g.cells) return;
  if (solid && solid[cell]) {
    if (n_) n_[cell] = 0.0;
    if (eps_) eps_[cell] = 0.0;
    if (P_) P_[cell] = 0.0;
    if (U_)
      for (int k = 0; k < 4; ++k) U_[k * g.cells + cell] = 0.0;
    return;
  }
  int x, y, z;
  cell_coords(cell, g, x, y, z);
  const Shifts sh(x, y, z, g);
  S f[M::Q];
  gather<M>(cur, g, sh, f, mode, cell);
  const Moments m = moments<M>(f);
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

// ---- solid walls: link-wise bounce-back ------------------------------------
//
// A population i whose source cell s = x - theta_i is solid must arrive at
// fluid cell x as the post-collision value of the inverse population at x.
// In the pull storage the next step reads population i of x from slot
// (i, s), so after each step the slot of the solid cell receives that value:
// nxt[i][s] = nxt[inv(i)][x] (inv(i) = i ^ 1).  Solid cells are never
// stored by the step kernels, so these slots are free; the written slots
// (solid cells) and the read slots (fluid cells) never overlap.
struct Link {
  int32_t dst; // solid cell s
  int32_t src; // fluid cell x = s + theta_pop
  int32_t pop; // population i
};

template <class M, class S>
__global__ void __launch_bounds__(BLOCK) k_bounce(S *__restrict__ nxt, const Link *__restrict__ links,
                                                  int64_t nlinks) {
  constexpr int T = TILE<S>;
  const int64_t k = static_cast<int64_t>(blockIdx.x) * BLOCK + threadIdx.x;
  if (k >= nlinks) return;
  const Link l = links[k];
  nxt[l.pop * T + tile_elem<M, S>(l.dst)] = nxt[(l.pop ^ 1) * T + tile_elem<M, S>(l.src)];
}

// Per-cell N^0 and T^{0 nu} of the current state (zero at solid cells):
// out[k * cells + cell] for k = N^0, T^00, T^0x, T^0y, T^0z.  With walls the
// per-population totals of k_popsum no longer give the box totals (solid
// slots hold copies), so the totals are summed per cell instead.
template <class M, class S>
__global__ void __launch_bounds__(BLOCK) k_cell_conserved(const S *__restrict__ cur, Geom g,
                                                          const uint8_t *__restrict__ solid,
                                                          double *__restrict__ out) {
  const int cell = blockIdx.x * BLOCK + threadIdx.x;
  if (cell >= g.cells) return;
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (!solid[cell]) {
    int x, y, z;
    cell_coords(cell, g, x, y, z);
    const Shifts sh(x, y, z, g);
    S f[M::Q];
    gather<M>(cur, g, sh, f);
    const Moments m = moments<M>(f);
    v[0] = m.N0;
    v[1] = m.T00;
    v[2] = m.T0x;
    v[3] = m.T0y;
    v[4] = m.T0z;
  }
  for (int k = 0; k < 5; ++k) out[static_cast<int64_t>(k) * g.cells + cell] = v[k];
}

// Per-population sums over all cells (streaming keeps each of them), in a
// fixed order: pass 1 writes one partial per (population, block) with a
// tree reduction over the block; pass 2 reduces the partials of each
// population the same way.
inline constexpr int SUM_CELLS_PER_THREAD = 16;

// The values summed: population i of the tiled storage (TILED), or row i
// of `cells` plain values `stride` apart.
template <class M, class S, bool TILED>
__global__ void __launch_bounds__(BLOCK) k_popsum_partial(const S *__restrict__ cur, Geom g, int64_t stride,
                                                          double *__restrict__ partial, int nblocks) {
  __shared__ double red[BLOCK];
  const int i = blockIdx.y;
  const S *base = cur + (TILED ? static_cast<int64_t>(i) * TILE<S> : i * stride);
  const int chunk = BLOCK * SUM_CELLS_PER_THREAD;
  const int c0 = blockIdx.x * chunk;
  double acc = 0.0;
  for (int j = 0; j < SUM_CELLS_PER_THREAD; ++j) {
    const int c = c0 + j * BLOCK + threadIdx.x;
    if (c < g.cells) acc += static_cast<double>(base[TILED ? tile_elem<M, S>(c) : c]);
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
