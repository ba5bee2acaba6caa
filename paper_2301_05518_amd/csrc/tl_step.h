// Smearing step kernels (eq. tlSmear with eq. tlLapl1) for gfx950, per right-hand side r:
//   out_r(x) = alpha in_r(x) + beta sum_mu [W_mu(x) in_r(x+2mu^) + W_mu^dag(x-2mu^) in_r(x-2mu^)]
// with alpha = 1 - 6 sigma/(4n) and beta = sigma/(4n), which is
// in + (sigma/n) Lap in.  (alpha = -3/2, beta = 1/4 gives Lap itself.)
// The RHS of one group live on the same slice and share every two-link load.
// Accumulation order per site is fixed (x fwd, x bwd, y fwd, y bwd, z fwd,
// z bwd, then the axpy), written with explicit fused multiply-adds, so every
// kernel variant and tiling produces bit-identical results.
//
// Included by one translation unit per storage precision (tl_step_<prec>.hip),
// each instantiating both two-link forms of its precision.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "tl_format.h"
#include "tl_internal.h"

namespace tl {

namespace {

constexpr int kXcds = 8;   // MI355X: 8 accelerator complex dies, each with its own L2

// Workgroups are dispatched round-robin over the XCDs (workgroup b runs on
// XCD b % 8).  Give the workgroups of one XCD a contiguous range of the work
// list and let them sweep it together, so neighbouring tiles (which share
// halo sites and two-links) meet in the same L2.  Correctness does not
// depend on the dispatch order.  rev: visit this workgroup's tiles in the
// opposite order (steps alternate, see StepConfig::flip).
struct TileSweep {
  int first, stride, n;
  bool rev;
  __device__ __forceinline__ int tile(int m) const { return first + (rev ? n - 1 - m : m) * stride; }
};

__device__ __forceinline__ TileSweep xcd_sweep(int n_tiles, int rev) {
  const int G = gridDim.x, b = blockIdx.x;
  const int k = b % kXcds, j = b / kXcds;
  const int q = G / kXcds, r = G % kXcds;
  const int cnt = q + (k < r ? 1 : 0);                     // workgroups on this XCD
  const int ord0 = k < r ? k * (q + 1) : r * (q + 1) + (k - r) * q;  // their first ordinal
  const int t0 = (int)(((int64_t)n_tiles * ord0) / G);
  const int t1 = (int)(((int64_t)n_tiles * (ord0 + cnt)) / G);
  const int first = t0 + j;
  return {first, cnt, first < t1 ? (t1 - first + cnt - 1) / cnt : 0, rev != 0};
}

// v mod L for v in [-2L, 3L), branch-free
__device__ __forceinline__ int wrap_sel(int v, int L) {
  v = v >= L ? v - L : v;
  v = v >= L ? v - L : v;
  v = v < 0 ? v + L : v;
  v = v < 0 ? v + L : v;
  return v;
}

__device__ __forceinline__ int wrap_step(int v, int d, int L) {
  v += d;
  while (v >= L) v -= L;
  while (v < 0) v += L;
  return v;
}

// acc += M v   (3x3 complex times colour vector)
template <typename T>
__device__ __forceinline__ void mv_acc(const T (&m)[18], const T (&v)[6], T (&acc)[6]) {
#pragma unroll
  for (int a = 0; a < 3; a++) {
    T re = acc[2 * a], im = acc[2 * a + 1];
#pragma unroll
    for (int b = 0; b < 3; b++) {
      const T mr = m[2 * (3 * a + b)], mi = m[2 * (3 * a + b) + 1];
      re = fma_(mr, v[2 * b], re);
      re = fma_(-mi, v[2 * b + 1], re);
      im = fma_(mr, v[2 * b + 1], im);
      im = fma_(mi, v[2 * b], im);
    }
    acc[2 * a] = re;
    acc[2 * a + 1] = im;
  }
}

// acc += M^dag v
template <typename T>
__device__ __forceinline__ void mdv_acc(const T (&m)[18], const T (&v)[6], T (&acc)[6]) {
#pragma unroll
  for (int a = 0; a < 3; a++) {
    T re = acc[2 * a], im = acc[2 * a + 1];
#pragma unroll
    for (int b = 0; b < 3; b++) {
      const T mr = m[2 * (3 * b + a)], mi = m[2 * (3 * b + a) + 1];
      re = fma_(mr, v[2 * b], re);
      re = fma_(mi, v[2 * b + 1], re);
      im = fma_(mr, v[2 * b + 1], im);
      im = fma_(-mi, v[2 * b], im);
    }
    acc[2 * a] = re;
    acc[2 * a + 1] = im;
  }
}

__device__ __forceinline__ int find_group(const StepGroup* __restrict__ groups, int n_groups, int tile) {
  int lo = 0, hi = n_groups - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (groups[mid].tile_begin <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------------------------------ step kernels

// Variant 0: each thread owns one (x, y) site of the tile and walks the tile's
// z planes; every neighbour value comes through L1/L2.
template <int P, int R, bool NT>
__global__ __launch_bounds__(256) void step_direct(const StepGroup* __restrict__ groups, int n_groups,
                                                   int tile_base, int n_tiles, int tz, int rev,
                                                   const char* __restrict__ in, char* __restrict__ out,
                                                   typename Fmt<P>::real alpha, typename Fmt<P>::real beta) {
  using F = Fmt<P>;
  using real = typename F::real;
  constexpr int D = hop_of(P);   // hop distance: 2 (two-link field), 1 (one-link field)
  constexpr int VB = kVBytes[P];
  (void)VB;
  const TileSweep sw = xcd_sweep(n_tiles, rev);
  for (int m = 0; m < sw.n; m++) {
    const int tl = sw.tile(m);
    const int tile = tile_base + tl;
    const StepGroup& g = groups[find_group(groups, n_groups, tile)];
    const int Lx = g.Lx, Ly = g.Ly, Lz = g.Lz;
    const int64_t Vp = g.Vp;
    const int local = tile - g.tile_begin;
    const int tzi = local / g.n_xy_tiles;
    const int txy = local - tzi * g.n_xy_tiles;
    const int LxLy = Lx * Ly;
    const int xy = txy * (int)blockDim.x + (int)threadIdx.x;
    if (xy >= LxLy) continue;
    const int y = xy / Lx, x = xy - y * Lx;
    const int xyp[2] = {y * Lx + wrap_step(x, D, Lx), wrap_step(y, D, Ly) * Lx + x};    // +D in x, y
    const int xym[2] = {y * Lx + wrap_step(x, -D, Lx), wrap_step(y, -D, Ly) * Lx + x};  // -D in x, y
    const char* Wmu[3] = {g.W, g.W + g.w_mu_stride, g.W + 2 * g.w_mu_stride};
    const int nr = g.nr;
    // Slots r >= nr of a narrower group read RHS nr-1 and store nothing: every load
    // is unconditional, so the compiler can keep many loads in flight.
    const char* pin[R];
    char* pout[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
      const int64_t o = g.psi_off + (int64_t)min(r, nr - 1) * g.rhs_stride;
      pin[r] = in + o;
      pout[r] = out + o;
    }
    const int z0 = tzi * tz;
    const int z1 = min(z0 + tz, Lz);
    for (int z = z0; z < z1; z++) {
      const int64_t zo = (int64_t)z * LxLy;
      const int64_t zp = (int64_t)wrap_step(z, D, Lz) * LxLy;
      const int64_t zm = (int64_t)wrap_step(z, -D, Lz) * LxLy;
      const int64_t site = zo + xy;
      const int64_t fwd[3] = {zo + xyp[0], zo + xyp[1], zp + xy};
      const int64_t bwd[3] = {zo + xym[0], zo + xym[1], zm + xy};
      real acc[R][6];
#pragma unroll
      for (int r = 0; r < R; r++)
#pragma unroll
        for (int c = 0; c < 6; c++) acc[r][c] = (real)0;
#pragma unroll
      for (int mu = 0; mu < 3; mu++) {
        real m[18];
        F::load_w(Wmu[mu], Vp, site, m);
#pragma unroll
        for (int r = 0; r < R; r++) {
          real v[6];
          F::load_v(pin[r], Vp, fwd[mu], v);
          mv_acc(m, v, acc[r]);
        }
        F::load_w(Wmu[mu], Vp, bwd[mu], m);
#pragma unroll
        for (int r = 0; r < R; r++) {
          real v[6];
          F::load_v(pin[r], Vp, bwd[mu], v);
          mdv_acc(m, v, acc[r]);
        }
      }
#pragma unroll
      for (int r = 0; r < R; r++) {
        real v[6], o[6];
        F::load_v(pin[r], Vp, site, v);
#pragma unroll
        for (int c = 0; c < 6; c++) o[c] = fma_(beta, acc[r][c], alpha * v[c]);
        if (r < nr) F::template store_v<real, NT>(pout[r], Vp, site, o);
      }
    }
  }
}

// Variant 1: as variant 0, but each thread keeps the colour vectors of planes
// z-2 .. z+2 in a register ring while it marches up the tile's z range, so the
// z hops and the centre term read no memory; one new plane is loaded per step.
template <int P, int R, bool NT>
__global__ __launch_bounds__(256) void step_zmarch(const StepGroup* __restrict__ groups, int n_groups,
                                                   int tile_base, int n_tiles, int tz, int rev,
                                                   const char* __restrict__ in, char* __restrict__ out,
                                                   typename Fmt<P>::real alpha, typename Fmt<P>::real beta) {
  using F = Fmt<P>;
  using real = typename F::real;
  const TileSweep sw = xcd_sweep(n_tiles, rev);
  for (int m = 0; m < sw.n; m++) {
    const int tl = sw.tile(m);
    const int tile = tile_base + tl;
    const StepGroup& g = groups[find_group(groups, n_groups, tile)];
    const int Lx = g.Lx, Ly = g.Ly, Lz = g.Lz;
    const int64_t Vp = g.Vp;
    const int local = tile - g.tile_begin;
    const int tzi = local / g.n_xy_tiles;
    const int txy = local - tzi * g.n_xy_tiles;
    const int LxLy = Lx * Ly;
    const int xy = txy * (int)blockDim.x + (int)threadIdx.x;
    if (xy >= LxLy) continue;
    const int y = xy / Lx, x = xy - y * Lx;
    const int xyp[2] = {y * Lx + wrap_step(x, 2, Lx), wrap_step(y, 2, Ly) * Lx + x};
    const int xym[2] = {y * Lx + wrap_step(x, -2, Lx), wrap_step(y, -2, Ly) * Lx + x};
    const char* Wmu[3] = {g.W, g.W + g.w_mu_stride, g.W + 2 * g.w_mu_stride};
    const int nr = g.nr;
    // Slots r >= nr of a narrower group read RHS nr-1 and store nothing: every load
    // is unconditional, so the compiler can keep many loads in flight.
    const char* pin[R];
    char* pout[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
      const int64_t o = g.psi_off + (int64_t)min(r, nr - 1) * g.rhs_stride;
      pin[r] = in + o;
      pout[r] = out + o;
    }
    const int z0 = tzi * tz;
    const int z1 = min(z0 + tz, Lz);
    real ring[5][R][6];   // planes z-2, z-1, z, z+1, z+2
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const int64_t zo = (int64_t)wrap_step(z0, k - 2, Lz) * LxLy + xy;
#pragma unroll
      for (int r = 0; r < R; r++)
        F::load_v(pin[r], Vp, zo, ring[k][r]);
    }
    for (int z = z0; z < z1; z++) {
      const int64_t zo = (int64_t)z * LxLy;
      const int64_t site = zo + xy;
      const int64_t zp = (int64_t)wrap_step(z, 2, Lz) * LxLy + xy;
      const int64_t zm = (int64_t)wrap_step(z, -2, Lz) * LxLy + xy;
#pragma unroll
      for (int r = 0; r < R; r++)
        F::load_v(pin[r], Vp, zp, ring[4][r]);
      real acc[R][6];
#pragma unroll
      for (int r = 0; r < R; r++)
#pragma unroll
        for (int c = 0; c < 6; c++) acc[r][c] = (real)0;
#pragma unroll
      for (int mu = 0; mu < 2; mu++) {
        real m[18];
        F::load_w(Wmu[mu], Vp, site, m);
#pragma unroll
        for (int r = 0; r < R; r++) {
          real v[6];
          F::load_v(pin[r], Vp, zo + xyp[mu], v);
          mv_acc(m, v, acc[r]);
        }
        F::load_w(Wmu[mu], Vp, zo + xym[mu], m);
#pragma unroll
        for (int r = 0; r < R; r++) {
          real v[6];
          F::load_v(pin[r], Vp, zo + xym[mu], v);
          mdv_acc(m, v, acc[r]);
        }
      }
      {
        real m[18];
        F::load_w(Wmu[2], Vp, site, m);
#pragma unroll
        for (int r = 0; r < R; r++)
          mv_acc(m, ring[4][r], acc[r]);
        F::load_w(Wmu[2], Vp, zm, m);
#pragma unroll
        for (int r = 0; r < R; r++)
          mdv_acc(m, ring[0][r], acc[r]);
      }
#pragma unroll
      for (int r = 0; r < R; r++) {
        real o[6];
#pragma unroll
        for (int c = 0; c < 6; c++) o[c] = fma_(beta, acc[r][c], alpha * ring[2][r][c]);
        if (r < nr) F::template store_v<real, NT>(pout[r], Vp, site, o);
      }
#pragma unroll
      for (int k = 0; k < 4; k++)
#pragma unroll
        for (int r = 0; r < R; r++)
#pragma unroll
          for (int c = 0; c < 6; c++) ring[k][r][c] = ring[k + 1][r][c];
    }
  }
}

// Variant 2: z-marching with register rings for both the colour vectors of
// planes z-2 .. z+2 and the z two-links of planes z-2 .. z, so every z hop
// and the centre term read no memory and each W_z is loaded once.  Even
// z chunks march up and odd chunks march down: two neighbouring chunks reach
// the planes they share at the same time, so those halo planes are still in
// L2 for the second reader.
template <int P, int R, bool NT>
__global__ __launch_bounds__(256) void step_zring(const StepGroup* __restrict__ groups, int n_groups,
                                                  int tile_base, int n_tiles, int tz, int rev,
                                                  const char* __restrict__ in, char* __restrict__ out,
                                                  typename Fmt<P>::real alpha, typename Fmt<P>::real beta) {
  using F = Fmt<P>;
  using real = typename F::real;
  const TileSweep sw = xcd_sweep(n_tiles, rev);
  for (int m = 0; m < sw.n; m++) {
    const int tl = sw.tile(m);
    const int tile = tile_base + tl;
    const StepGroup& g = groups[find_group(groups, n_groups, tile)];
    const int Lx = g.Lx, Ly = g.Ly, Lz = g.Lz;
    const int64_t Vp = g.Vp;
    const int local = tile - g.tile_begin;
    const int tzi = local / g.n_xy_tiles;
    const int txy = local - tzi * g.n_xy_tiles;
    const int LxLy = Lx * Ly;
    const int xy = txy * (int)blockDim.x + (int)threadIdx.x;
    if (xy >= LxLy) continue;
    const int y = xy / Lx, x = xy - y * Lx;
    const int xyp[2] = {y * Lx + wrap_step(x, 2, Lx), wrap_step(y, 2, Ly) * Lx + x};
    const int xym[2] = {y * Lx + wrap_step(x, -2, Lx), wrap_step(y, -2, Ly) * Lx + x};
    const char* Wmu[3] = {g.W, g.W + g.w_mu_stride, g.W + 2 * g.w_mu_stride};
    const int nr = g.nr;
    // Slots r >= nr of a narrower group read RHS nr-1 and store nothing: every load
    // is unconditional, so the compiler can keep many loads in flight.
    const char* pin[R];
    char* pout[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
      const int64_t o = g.psi_off + (int64_t)min(r, nr - 1) * g.rhs_stride;
      pin[r] = in + o;
      pout[r] = out + o;
    }
    const int zlo = tzi * tz;
    const int nz = min(zlo + tz, Lz) - zlo;
    const bool up = ((tzi & 1) == 0) != (rev != 0);
    const int dz = up ? 1 : -1;
    const int zs = up ? zlo : zlo + nz - 1;       // first plane of the march
    // ring[k] holds plane zs + dz*(k-2) relative to the current plane, i.e. k = 2 is
    // the current plane and k = 4 the one two planes ahead in the march direction.
    real ring[5][R][6];
    // Each step loads one new W_z into wz[2]: W_z(z) marching up, W_z(z-2) marching
    // down; wz[k] was loaded 2-k steps earlier.  So wz[k] = W_z(z-2+k) marching up
    // and W_z(z-k) marching down: both hops' two-links are wz[0] and wz[2].
    real wz[3][18];
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const int64_t zo = (int64_t)wrap_step(zs, dz * (k - 2), Lz) * LxLy + xy;
#pragma unroll
      for (int r = 0; r < R; r++)
        F::load_v(pin[r], Vp, zo, ring[k][r]);
    }
#pragma unroll
    for (int k = 0; k < 2; k++) {
      const int64_t zo = (int64_t)wrap_step(zs, up ? k - 2 : -k, Lz) * LxLy + xy;
      F::load_w(Wmu[2], Vp, zo, wz[k]);
    }
    for (int i = 0; i < nz; i++) {
      const int z = zs + dz * i;
      const int64_t zo = (int64_t)z * LxLy;
      const int64_t site = zo + xy;
      {
        const int64_t za = (int64_t)wrap_step(z, 2 * dz, Lz) * LxLy + xy;   // two planes ahead
#pragma unroll
        for (int r = 0; r < R; r++)
          F::load_v(pin[r], Vp, za, ring[4][r]);
        // marching up the new W_z is the current plane's (forward hop); marching down it is the
        // plane two below (backward hop)
        const int64_t zw = up ? site : (int64_t)wrap_step(z, -2, Lz) * LxLy + xy;
        F::load_w(Wmu[2], Vp, zw, wz[2]);
      }
      real acc[R][6];
#pragma unroll
      for (int r = 0; r < R; r++)
#pragma unroll
        for (int c = 0; c < 6; c++) acc[r][c] = (real)0;
#pragma unroll
      for (int mu = 0; mu < 2; mu++) {
        real m[18];
        F::load_w(Wmu[mu], Vp, site, m);
#pragma unroll
        for (int r = 0; r < R; r++) {
          real v[6];
          F::load_v(pin[r], Vp, zo + xyp[mu], v);
          mv_acc(m, v, acc[r]);
        }
        F::load_w(Wmu[mu], Vp, zo + xym[mu], m);
#pragma unroll
        for (int r = 0; r < R; r++) {
          real v[6];
          F::load_v(pin[r], Vp, zo + xym[mu], v);
          mdv_acc(m, v, acc[r]);
        }
      }
      // z forward: W_z(z) psi(z+2); z backward: W_z(z-2)^dag psi(z-2)
      if (up) {
#pragma unroll
        for (int r = 0; r < R; r++)
          mv_acc(wz[2], ring[4][r], acc[r]);
#pragma unroll
        for (int r = 0; r < R; r++)
          mdv_acc(wz[0], ring[0][r], acc[r]);
      } else {
#pragma unroll
        for (int r = 0; r < R; r++)
          mv_acc(wz[0], ring[0][r], acc[r]);
#pragma unroll
        for (int r = 0; r < R; r++)
          mdv_acc(wz[2], ring[4][r], acc[r]);
      }
#pragma unroll
      for (int r = 0; r < R; r++) {
        real o[6];
#pragma unroll
        for (int c = 0; c < 6; c++) o[c] = fma_(beta, acc[r][c], alpha * ring[2][r][c]);
        if (r < nr) F::template store_v<real, NT>(pout[r], Vp, site, o);
      }
#pragma unroll
      for (int k = 0; k < 4; k++)
#pragma unroll
        for (int r = 0; r < R; r++)
#pragma unroll
          for (int c = 0; c < 6; c++) ring[k][r][c] = ring[k + 1][r][c];
#pragma unroll
      for (int c = 0; c < 18; c++) {
        wz[0][c] = wz[1][c];
        wz[1][c] = wz[2][c];
      }
    }
  }
}

// In-plane hops (x forward, x backward, y forward, y backward, in that order)
// of the site xy of plane zo, for every RHS slot.
template <class F, int R, typename real>
__device__ __forceinline__ void inplane_hops(const char* const (&Wmu)[3], const char* const (&pin)[R], int64_t Vp,
                                             int64_t zo, int xy, const int (&xyp)[2], const int (&xym)[2],
                                             real (&acc)[R][6]) {
#pragma unroll
  for (int r = 0; r < R; r++)
#pragma unroll
    for (int c = 0; c < 6; c++) acc[r][c] = (real)0;
#pragma unroll
  for (int mu = 0; mu < 2; mu++) {
    real m[18];
    F::load_w(Wmu[mu], Vp, zo + xy, m);
#pragma unroll
    for (int r = 0; r < R; r++) {
      real v[6];
      F::load_v(pin[r], Vp, zo + xyp[mu], v);
      mv_acc(m, v, acc[r]);
    }
    F::load_w(Wmu[mu], Vp, zo + xym[mu], m);
#pragma unroll
    for (int r = 0; r < R; r++) {
      real v[6];
      F::load_v(pin[r], Vp, zo + xym[mu], v);
      mdv_acc(m, v, acc[r]);
    }
  }
}

// Variant 3: z-marching in which every plane is read from memory once, at
// the front of the march.  When plane f = z+2 is first touched, the thread
// loads its own colour vectors there (register ring of planes z-2 .. z+2)
// and also computes the in-plane hops of plane f, whose neighbour rows the
// workgroup and its y-neighbour workgroups are loading in the same step, so
// they come from L2.  Those partial sums wait in a ring for two steps; at
// plane z the two z hops (W_z from a register ring) and the axpy complete
// the site.  Chunks alternate their march direction as in variant 2.
template <int P, int R, bool NT>
__global__ __launch_bounds__(256) void step_zfront(const StepGroup* __restrict__ groups, int n_groups,
                                                   int tile_base, int n_tiles, int tz, int rev,
                                                   const char* __restrict__ in, char* __restrict__ out,
                                                   typename Fmt<P>::real alpha, typename Fmt<P>::real beta) {
  using F = Fmt<P>;
  using real = typename F::real;
  const TileSweep sw = xcd_sweep(n_tiles, rev);
  for (int m = 0; m < sw.n; m++) {
    const int tl = sw.tile(m);
    const int tile = tile_base + tl;
    const StepGroup& g = groups[find_group(groups, n_groups, tile)];
    const int Lx = g.Lx, Ly = g.Ly, Lz = g.Lz;
    const int64_t Vp = g.Vp;
    const int local = tile - g.tile_begin;
    const int tzi = local / g.n_xy_tiles;
    const int txy = local - tzi * g.n_xy_tiles;
    const int LxLy = Lx * Ly;
    const int xy = txy * (int)blockDim.x + (int)threadIdx.x;
    if (xy >= LxLy) continue;
    const int y = xy / Lx, x = xy - y * Lx;
    const int xyp[2] = {y * Lx + wrap_step(x, 2, Lx), wrap_step(y, 2, Ly) * Lx + x};
    const int xym[2] = {y * Lx + wrap_step(x, -2, Lx), wrap_step(y, -2, Ly) * Lx + x};
    const char* const Wmu[3] = {g.W, g.W + g.w_mu_stride, g.W + 2 * g.w_mu_stride};
    const int nr = g.nr;
    const char* pin[R];
    char* pout[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
      const int64_t o = g.psi_off + (int64_t)min(r, nr - 1) * g.rhs_stride;
      pin[r] = in + o;
      pout[r] = out + o;
    }
    const int zlo = tzi * tz;
    const int nz = min(zlo + tz, Lz) - zlo;
    const bool up = ((tzi & 1) == 0) != (rev != 0);
    const int dz = up ? 1 : -1;
    const int zs = up ? zlo : zlo + nz - 1;
    real ring[5][R][6];      // own colour vectors, planes z-2dz .. z+2dz
    real part[2][R][6];      // in-plane partial sums of planes z and z+dz
    real wz[3][18];          // as in variant 2: wz[0], wz[2] are the two z hops' links
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const int64_t zo = (int64_t)wrap_step(zs, dz * (k - 2), Lz) * LxLy + xy;
#pragma unroll
      for (int r = 0; r < R; r++) F::load_v(pin[r], Vp, zo, ring[k][r]);
    }
#pragma unroll
    for (int k = 0; k < 2; k++) {
      const int64_t zw = (int64_t)wrap_step(zs, up ? k - 2 : -k, Lz) * LxLy + xy;
      F::load_w(Wmu[2], Vp, zw, wz[k]);
      const int64_t zp = (int64_t)wrap_step(zs, dz * k, Lz) * LxLy;
      if (k < nz) inplane_hops<F, R>(Wmu, pin, Vp, zp, xy, xyp, xym, part[k]);
    }
    for (int i = 0; i < nz; i++) {
      const int z = zs + dz * i;
      const int64_t zo = (int64_t)z * LxLy;
      const int64_t site = zo + xy;
      const int64_t zf = (int64_t)wrap_step(z, 2 * dz, Lz) * LxLy;   // front plane
#pragma unroll
      for (int r = 0; r < R; r++) F::load_v(pin[r], Vp, zf + xy, ring[4][r]);
      F::load_w(Wmu[2], Vp, up ? site : (int64_t)wrap_step(z, -2, Lz) * LxLy + xy, wz[2]);
      real front[R][6];
      if (i + 2 < nz) inplane_hops<F, R>(Wmu, pin, Vp, zf, xy, xyp, xym, front);
      // complete plane z: in-plane part, then z forward, then z backward, then the axpy
      const real (&fw)[18] = up ? wz[2] : wz[0];
      const real (&bw)[18] = up ? wz[0] : wz[2];
#pragma unroll
      for (int r = 0; r < R; r++) {
        mv_acc(fw, up ? ring[4][r] : ring[0][r], part[0][r]);
        mdv_acc(bw, up ? ring[0][r] : ring[4][r], part[0][r]);
        real o[6];
#pragma unroll
        for (int c = 0; c < 6; c++) o[c] = fma_(beta, part[0][r][c], alpha * ring[2][r][c]);
        if (r < nr) F::template store_v<real, NT>(pout[r], Vp, site, o);
      }
#pragma unroll
      for (int k = 0; k < 4; k++)
#pragma unroll
        for (int r = 0; r < R; r++)
#pragma unroll
          for (int c = 0; c < 6; c++) ring[k][r][c] = ring[k + 1][r][c];
#pragma unroll
      for (int c = 0; c < 18; c++) {
        wz[0][c] = wz[1][c];
        wz[1][c] = wz[2][c];
      }
#pragma unroll
      for (int r = 0; r < R; r++)
#pragma unroll
        for (int c = 0; c < 6; c++) {
          part[0][r][c] = part[1][r][c];
          part[1][r][c] = front[r][c];
        }
    }
  }
}

// Variant 4: as variant 0, but the loop over directions stays rolled, so only
// one direction's loads (two two-links and 2R colour vectors) are live at a
// time.  Fewer registers allow more waves per SIMD, which hide the memory
// latency of each direction and overlap one wave's arithmetic with the
// others' loads.  Fields are addressed through per-plane base pointers (uniform
// across the workgroup) plus 32-bit site offsets, so a load costs one offset
// rather than a 64-bit address computation.
template <int P, int R, bool NT>
__global__ __launch_bounds__(256) void step_rolled(const StepGroup* __restrict__ groups, int n_groups,
                                                   int tile_base, int n_tiles, int tz, int rev,
                                                   const char* __restrict__ in, char* __restrict__ out,
                                                   typename Fmt<P>::real alpha, typename Fmt<P>::real beta) {
  using PL = Planes<P>;
  using real = typename Fmt<P>::real;
  constexpr int D = hop_of(P);   // hop distance: 2 (two-link field), 1 (one-link field)
  const TileSweep sw = xcd_sweep(n_tiles, rev);
  for (int m = 0; m < sw.n; m++) {
    const int tl = sw.tile(m);
    const int tile = tile_base + tl;
    const StepGroup& g = groups[find_group(groups, n_groups, tile)];
    const int Lx = g.Lx, Ly = g.Ly, Lz = g.Lz;
    const int64_t Vp = g.Vp;
    const int local = tile - g.tile_begin;
    const int tzi = local / g.n_xy_tiles;
    const int txy = local - tzi * g.n_xy_tiles;
    const int LxLy = Lx * Ly;
    const int xy = txy * (int)blockDim.x + (int)threadIdx.x;
    if (xy >= LxLy) continue;
    const int y = xy / Lx, x = xy - y * Lx;
    const int xf = y * Lx + wrap_step(x, D, Lx), xb = y * Lx + wrap_step(x, -D, Lx);
    const int yf = wrap_step(y, D, Ly) * Lx + x, yb = wrap_step(y, -D, Ly) * Lx + x;
    const int nr = g.nr;
    const char* ip[R][PL::NV];
    char* op[R][PL::NV];
#pragma unroll
    for (int r = 0; r < R; r++) {
      const int64_t o = g.psi_off + (int64_t)min(r, nr - 1) * g.rhs_stride;
      PL::v(in + o, Vp, ip[r]);
      PL::v(out + o, Vp, op[r]);
    }
    const int z0 = tzi * tz;
    const int z1 = min(z0 + tz, Lz);
    for (int z = z0; z < z1; z++) {
      const uint32_t zo = (uint32_t)(z * LxLy);
      const uint32_t zf = (uint32_t)(wrap_sel(z + D, Lz) * LxLy + xy);
      const uint32_t zb = (uint32_t)(wrap_sel(z - D, Lz) * LxLy + xy);
      const uint32_t site = zo + (uint32_t)xy;
      real acc[R][6];
#pragma unroll
      for (int r = 0; r < R; r++)
#pragma unroll
        for (int c = 0; c < 6; c++) acc[r][c] = (real)0;
#pragma unroll 1
      for (int mu = 0; mu < 3; mu++) {
        const char* wp[PL::NW];
        PL::w(g.W + mu * g.w_mu_stride, Vp, wp);
        const uint32_t f = mu == 0 ? zo + (uint32_t)xf : (mu == 1 ? zo + (uint32_t)yf : zf);
        const uint32_t b = mu == 0 ? zo + (uint32_t)xb : (mu == 1 ? zo + (uint32_t)yb : zb);
        real mtx[18];
        PL::load_w(wp, site, mtx);
#pragma unroll
        for (int r = 0; r < R; r++) {
          real v[6];
          PL::load_v(ip[r], f, v);
          mv_acc(mtx, v, acc[r]);
        }
        PL::load_w(wp, b, mtx);
#pragma unroll
        for (int r = 0; r < R; r++) {
          real v[6];
          PL::load_v(ip[r], b, v);
          mdv_acc(mtx, v, acc[r]);
        }
      }
#pragma unroll
      for (int r = 0; r < R; r++) {
        real v[6], o[6];
        PL::load_v(ip[r], site, v);
#pragma unroll
        for (int c = 0; c < 6; c++) o[c] = fma_(beta, acc[r][c], alpha * v[c]);
        if (r < nr) PL::template store_v<real, NT>(op[r], site, o);
      }
    }
  }
}

template <typename T> struct Complex2;
template <> struct Complex2<float> { using type = float2; };
template <> struct Complex2<double> { using type = double2; };

// Variant 5: z-marching as variant 2 (register rings of colour vectors and z
// two-links, alternating chunk directions) on tiles of `rows` full rows of the
// xy plane.  Each step every thread publishes its current-plane colour vectors
// to LDS and the first 4*Lx threads load the four halo rows (two above, two
// below, periodic); all in-plane neighbours are then read from LDS.  Two LDS
// buffers alternate by step, so one barrier per step suffices.  Threads past
// the tile's rows only help with the barrier and the halo.  Fields are
// addressed through per-plane base pointers set up once per tile and 32-bit
// site offsets; plane wraps are branch-free.
template <int P, int R, bool NT>
__global__ __launch_bounds__(512) void step_zlds(const StepGroup* __restrict__ groups, int n_groups,
                                                 int tile_base, int n_tiles, int tz, int rev,
                                                 const char* __restrict__ in, char* __restrict__ out,
                                                 typename Fmt<P>::real alpha, typename Fmt<P>::real beta) {
  using PL = Planes<P>;
  using real = typename Fmt<P>::real;
  using c2 = typename Complex2<real>::type;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  c2* const lds = reinterpret_cast<c2*>(lds_raw);
  const TileSweep sw = xcd_sweep(n_tiles, rev);
  int it = 0;   // steps done by this workgroup: selects the LDS buffer across tiles
  for (int m = 0; m < sw.n; m++) {
    const int tl = sw.tile(m);
    const int tile = tile_base + tl;
    const StepGroup& g = groups[find_group(groups, n_groups, tile)];
    const int Lx = g.Lx, Ly = g.Ly, Lz = g.Lz, rows = g.rows;
    const int64_t Vp = g.Vp;
    const int local = tile - g.tile_begin;
    const int tzi = local / g.n_xy_tiles;
    const int y0 = (local - tzi * g.n_xy_tiles) * rows;
    const int LxLy = Lx * Ly;
    const int t = (int)threadIdx.x;
    const int trow = t / Lx, x = t - trow * Lx;
    const bool active = trow < rows;
    const int row = active ? trow : 0;
    const int y = y0 + row;
    const int xy = y * Lx + x;
    const int xbw = y * Lx + wrap_sel(x - 2, Lx);
    const int ybw = wrap_sel(y - 2, Ly) * Lx + x;
    const int nsite = (rows + 4) * Lx;
    const int own = (row + 2) * Lx + x;
    const int sxf = (row + 2) * Lx + wrap_sel(x + 2, Lx), sxb = (row + 2) * Lx + wrap_sel(x - 2, Lx);
    const int syf = (row + 4) * Lx + x, syb = row * Lx + x;
    const bool halo = t < 4 * Lx;
    const int hr = halo ? trow : 0;
    const int hrho = hr < 2 ? hr - 2 : rows + hr - 2;          // halo row relative to y0
    const int hxy = wrap_sel(y0 + hrho, Ly) * Lx + x;
    const int hslot = (hrho + 2) * Lx + x;
    const char* wp[3][PL::NW];
#pragma unroll
    for (int mu = 0; mu < 3; mu++) PL::w(g.W + mu * g.w_mu_stride, Vp, wp[mu]);
    const int nr = g.nr;
    const char* ip[R][PL::NV];
    char* op[R][PL::NV];
#pragma unroll
    for (int r = 0; r < R; r++) {
      const int64_t o = g.psi_off + (int64_t)min(r, nr - 1) * g.rhs_stride;
      PL::v(in + o, Vp, ip[r]);
      PL::v(out + o, Vp, op[r]);
    }
    const int zlo = tzi * tz;
    const int nz = min(zlo + tz, Lz) - zlo;
    const bool up = ((tzi & 1) == 0) != (rev != 0);
    const int dz = up ? 1 : -1;
    const int zs = up ? zlo : zlo + nz - 1;
    real ring[5][R][6];
    real wz[3][18];
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const uint32_t zo = (uint32_t)(wrap_sel(zs + dz * (k - 2), Lz) * LxLy + xy);
#pragma unroll
      for (int r = 0; r < R; r++) PL::load_v(ip[r], zo, ring[k][r]);
    }
#pragma unroll
    for (int k = 0; k < 2; k++)
      PL::load_w(wp[2], (uint32_t)(wrap_sel(zs + (up ? k - 2 : -k), Lz) * LxLy + xy), wz[k]);
    for (int i = 0; i < nz; i++, it++) {
      const int z = zs + dz * i;
      const uint32_t zo = (uint32_t)(z * LxLy);
      const uint32_t site = zo + xy;
      {
        const uint32_t za = (uint32_t)(wrap_sel(z + 2 * dz, Lz) * LxLy + xy);
#pragma unroll
        for (int r = 0; r < R; r++) PL::load_v(ip[r], za, ring[4][r]);
        const uint32_t zw = up ? site : (uint32_t)(wrap_sel(z - 2, Lz) * LxLy + xy);
        PL::load_w(wp[2], zw, wz[2]);
      }
      c2* const buf = lds + (it & 1) * (R * 3) * nsite;
      if (halo) {
#pragma unroll
        for (int r = 0; r < R; r++) {
          real hv[6];
          PL::load_v(ip[r], zo + hxy, hv);
#pragma unroll
          for (int c = 0; c < 3; c++) buf[(r * 3 + c) * nsite + hslot] = c2{hv[2 * c], hv[2 * c + 1]};
        }
      }
      if (active) {
#pragma unroll
        for (int r = 0; r < R; r++)
#pragma unroll
          for (int c = 0; c < 3; c++) buf[(r * 3 + c) * nsite + own] = c2{ring[2][r][2 * c], ring[2][r][2 * c + 1]};
      }
      __syncthreads();
      real acc[R][6];
#pragma unroll
      for (int r = 0; r < R; r++)
#pragma unroll
        for (int c = 0; c < 6; c++) acc[r][c] = (real)0;
#pragma unroll
      for (int mu = 0; mu < 2; mu++) {
        const int sf = mu == 0 ? sxf : syf, sb = mu == 0 ? sxb : syb;
        real m[18];
        PL::load_w(wp[mu], site, m);
#pragma unroll
        for (int r = 0; r < R; r++) {
          real v[6];
#pragma unroll
          for (int c = 0; c < 3; c++) {
            const c2 w = buf[(r * 3 + c) * nsite + sf];
            v[2 * c] = w.x;
            v[2 * c + 1] = w.y;
          }
          mv_acc(m, v, acc[r]);
        }
        PL::load_w(wp[mu], zo + (uint32_t)(mu == 0 ? xbw : ybw), m);
#pragma unroll
        for (int r = 0; r < R; r++) {
          real v[6];
#pragma unroll
          for (int c = 0; c < 3; c++) {
            const c2 w = buf[(r * 3 + c) * nsite + sb];
            v[2 * c] = w.x;
            v[2 * c + 1] = w.y;
          }
          mdv_acc(m, v, acc[r]);
        }
      }
      if (up) {
#pragma unroll
        for (int r = 0; r < R; r++) mv_acc(wz[2], ring[4][r], acc[r]);
#pragma unroll
        for (int r = 0; r < R; r++) mdv_acc(wz[0], ring[0][r], acc[r]);
      } else {
#pragma unroll
        for (int r = 0; r < R; r++) mv_acc(wz[0], ring[0][r], acc[r]);
#pragma unroll
        for (int r = 0; r < R; r++) mdv_acc(wz[2], ring[4][r], acc[r]);
      }
#pragma unroll
      for (int r = 0; r < R; r++) {
        real o[6];
#pragma unroll
        for (int c = 0; c < 6; c++) o[c] = fma_(beta, acc[r][c], alpha * ring[2][r][c]);
        if (active && r < nr) PL::template store_v<real, NT>(op[r], site, o);
      }
#pragma unroll
      for (int k = 0; k < 4; k++)
#pragma unroll
        for (int r = 0; r < R; r++)
#pragma unroll
          for (int c = 0; c < 6; c++) ring[k][r][c] = ring[k + 1][r][c];
#pragma unroll
      for (int c = 0; c < 18; c++) {
        wz[0][c] = wz[1][c];
        wz[1][c] = wz[2][c];
      }
    }
  }
}

// Variant 6: as variant 5, but each tile marches a chain of planes z, z+2,
// z+4, ... (mod Lz; two chains when Lz is even, one when odd), so the z hops
// are the chain neighbours: a ring of three colour-vector planes and two z
// two-links suffices.  The registers this frees hold the four in-plane
// two-links, which are loaded before the LDS barrier so their latency
// overlaps it.  Tiles: (row tile, chain, chunk of tz chain positions); chunks
// alternate their march direction along the chain.
template <int P, int R, bool NT>
__global__ __launch_bounds__(512) void step_zchain(const StepGroup* __restrict__ groups, int n_groups,
                                                   int tile_base, int n_tiles, int tz, int rev,
                                                   const char* __restrict__ in, char* __restrict__ out,
                                                   typename Fmt<P>::real alpha, typename Fmt<P>::real beta) {
  using PL = Planes<P>;
  using real = typename Fmt<P>::real;
  using c2 = typename Complex2<real>::type;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  c2* const lds = reinterpret_cast<c2*>(lds_raw);
  const TileSweep sw = xcd_sweep(n_tiles, rev);
  int it = 0;
  for (int m = 0; m < sw.n; m++) {
    const int tl = sw.tile(m);
    const int tile = tile_base + tl;
    const StepGroup& g = groups[find_group(groups, n_groups, tile)];
    const int Lx = g.Lx, Ly = g.Ly, Lz = g.Lz, rows = g.rows;
    const int64_t Vp = g.Vp;
    const int local = tile - g.tile_begin;
    const int tzi = local / g.n_xy_tiles;          // chain chunk index: n_z_tiles = chains * chunks
    const int y0 = (local - tzi * g.n_xy_tiles) * rows;
    const int chains = (Lz & 1) ? 1 : 2;
    const int clen = Lz / chains;                  // planes per chain
    const int chunks = (clen + tz - 1) / tz;
    const int chain = tzi / chunks, chunk = tzi - chain * chunks;
    const int LxLy = Lx * Ly;
    const int t = (int)threadIdx.x;
    const int trow = t / Lx, x = t - trow * Lx;
    const bool active = trow < rows;
    const int row = active ? trow : 0;
    const int y = y0 + row;
    const int xy = y * Lx + x;
    const int xbw = y * Lx + wrap_sel(x - 2, Lx);
    const int ybw = wrap_sel(y - 2, Ly) * Lx + x;
    const int nsite = (rows + 4) * Lx;
    const int own = (row + 2) * Lx + x;
    const int sxf = (row + 2) * Lx + wrap_sel(x + 2, Lx), sxb = (row + 2) * Lx + wrap_sel(x - 2, Lx);
    const int syf = (row + 4) * Lx + x, syb = row * Lx + x;
    const bool halo = t < 4 * Lx;
    const int hr = halo ? trow : 0;
    const int hrho = hr < 2 ? hr - 2 : rows + hr - 2;
    const int hxy = wrap_sel(y0 + hrho, Ly) * Lx + x;
    const int hslot = (hrho + 2) * Lx + x;
    const char* wp[3][PL::NW];
#pragma unroll
    for (int mu = 0; mu < 3; mu++) PL::w(g.W + mu * g.w_mu_stride, Vp, wp[mu]);
    const int nr = g.nr;
    const char* ip[R][PL::NV];
    char* op[R][PL::NV];
#pragma unroll
    for (int r = 0; r < R; r++) {
      const int64_t o = g.psi_off + (int64_t)min(r, nr - 1) * g.rhs_stride;
      PL::v(in + o, Vp, ip[r]);
      PL::v(out + o, Vp, op[r]);
    }
    const int k0 = chunk * tz;
    const int nz = min(k0 + tz, clen) - k0;        // planes of this chunk
    const bool up = ((chunk & 1) == 0) != (rev != 0);
    // first plane of the march: chain position k0 (up) or k0 + nz - 1 (down)
    const int kf = up ? k0 : k0 + nz - 1;
    int z = wrap_sel(chain + 2 * kf, Lz);          // kf < Lz, so the argument is below 3 Lz
    const int step = up ? 2 : -2;                  // plane step along the march
    // ring[0]: plane behind in the march, ring[1]: current, ring[2]: ahead (loaded each step)
    real ring[3][R][6];
    real wz[2][18];   // wz[0] loaded one step earlier, wz[1] this step
    {
      const uint32_t zb = (uint32_t)(wrap_sel(z - step, Lz) * LxLy + xy);
      const uint32_t zc = (uint32_t)(z * LxLy + xy);
#pragma unroll
      for (int r = 0; r < R; r++) {
        PL::load_v(ip[r], zb, ring[0][r]);
        PL::load_v(ip[r], zc, ring[1][r]);
      }
      // marching up the link loaded at plane z is W_z(z); marching down it is W_z(z-2),
      // so before the first step wz[0] holds W_z(z-2) (up) or W_z(z) (down)
      PL::load_w(wp[2], up ? (uint32_t)(wrap_sel(z - 2, Lz) * LxLy + xy) : zc, wz[0]);
    }
    for (int i = 0; i < nz; i++, it++) {
      const uint32_t zo = (uint32_t)(z * LxLy);
      const uint32_t site = zo + xy;
      const int za = wrap_sel(z + step, Lz);
#pragma unroll
      for (int r = 0; r < R; r++) PL::load_v(ip[r], (uint32_t)(za * LxLy + xy), ring[2][r]);
      PL::load_w_raw(wp[2], up ? site : (uint32_t)(wrap_sel(z - 2, Lz) * LxLy + xy), wz[1]);
      real mxf[18], mxb[18], myf[18], myb[18];
      PL::load_w_raw(wp[0], site, mxf);
      PL::load_w_raw(wp[0], zo + (uint32_t)xbw, mxb);
      PL::load_w_raw(wp[1], site, myf);
      PL::load_w_raw(wp[1], zo + (uint32_t)ybw, myb);
      c2* const buf = lds + (it & 1) * (R * 3) * nsite;
      if (halo) {
#pragma unroll
        for (int r = 0; r < R; r++) {
          real hv[6];
          PL::load_v(ip[r], zo + hxy, hv);
#pragma unroll
          for (int c = 0; c < 3; c++) buf[(r * 3 + c) * nsite + hslot] = c2{hv[2 * c], hv[2 * c + 1]};
        }
      }
      if (active) {
#pragma unroll
        for (int r = 0; r < R; r++)
#pragma unroll
          for (int c = 0; c < 3; c++) buf[(r * 3 + c) * nsite + own] = c2{ring[1][r][2 * c], ring[1][r][2 * c + 1]};
      }
      __syncthreads();
      PL::finish_w(wz[1]);
      PL::finish_w(mxf);
      PL::finish_w(mxb);
      PL::finish_w(myf);
      PL::finish_w(myb);
      real acc[R][6];
#pragma unroll
      for (int r = 0; r < R; r++) {
#pragma unroll
        for (int c = 0; c < 6; c++) acc[r][c] = (real)0;
        real v[6];
#pragma unroll
        for (int c = 0; c < 3; c++) { const c2 w = buf[(r * 3 + c) * nsite + sxf]; v[2 * c] = w.x; v[2 * c + 1] = w.y; }
        mv_acc(mxf, v, acc[r]);
#pragma unroll
        for (int c = 0; c < 3; c++) { const c2 w = buf[(r * 3 + c) * nsite + sxb]; v[2 * c] = w.x; v[2 * c + 1] = w.y; }
        mdv_acc(mxb, v, acc[r]);
#pragma unroll
        for (int c = 0; c < 3; c++) { const c2 w = buf[(r * 3 + c) * nsite + syf]; v[2 * c] = w.x; v[2 * c + 1] = w.y; }
        mv_acc(myf, v, acc[r]);
#pragma unroll
        for (int c = 0; c < 3; c++) { const c2 w = buf[(r * 3 + c) * nsite + syb]; v[2 * c] = w.x; v[2 * c + 1] = w.y; }
        mdv_acc(myb, v, acc[r]);
      }
      // z forward: W_z(z) psi(z+2); z backward: W_z(z-2)^dag psi(z-2)
      if (up) {
#pragma unroll
        for (int r = 0; r < R; r++) {
          mv_acc(wz[1], ring[2][r], acc[r]);
          mdv_acc(wz[0], ring[0][r], acc[r]);
        }
      } else {
#pragma unroll
        for (int r = 0; r < R; r++) {
          mv_acc(wz[0], ring[0][r], acc[r]);
          mdv_acc(wz[1], ring[2][r], acc[r]);
        }
      }
#pragma unroll
      for (int r = 0; r < R; r++) {
        real o[6];
#pragma unroll
        for (int c = 0; c < 6; c++) o[c] = fma_(beta, acc[r][c], alpha * ring[1][r][c]);
        if (active && r < nr) PL::template store_v<real, NT>(op[r], site, o);
      }
#pragma unroll
      for (int r = 0; r < R; r++)
#pragma unroll
        for (int c = 0; c < 6; c++) {
          ring[0][r][c] = ring[1][r][c];
          ring[1][r][c] = ring[2][r][c];
        }
#pragma unroll
      for (int c = 0; c < 18; c++) wz[0][c] = wz[1][c];
      z = za;
    }
  }
}

// Words of a two-link that load_w_raw fills before finish_w completes it: 18 (eighteen-real
// FP64, FP32 and F16S, the latter widened at load), 12 (twelve-real forms) or 9 (BF16, whose
// packed words are widened by finish_w).
constexpr int raw_words(int P) { return is_w12(P) ? 12 : ((P & 3) == BF16 ? 9 : 18); }

// Forms whose LDS-staged kernels take the backward x two-link from a neighbouring lane on
// rows of 64 sites: FP32 and eighteen-real F16S (the others would spill the registers the
// second code path needs).
constexpr bool lane_xbw(int P) { return (P & 3) == F32 || (P & 7) == F16S; }

// The value v of lane src of the wave (src in bytes: lane * 4).
__device__ __forceinline__ float lane_get(float v, int src) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(v)));
}
__device__ __forceinline__ double lane_get(double v, int src) {
  const int lo = __builtin_amdgcn_ds_bpermute(src, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(src, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

// Variant 7: variant 6 software-pipelined across plane steps.  The waves of a
// workgroup meet at the LDS barrier every step, so they all wait for memory at
// the same time unless a step's loads are issued a step early.  Each step
// therefore issues, right after its in-plane hops, the next plane's in-plane
// two-links and halo rows (into the registers those hops just freed), and right
// after its z hops the next plane's colour vectors ahead in the march and its z
// two-link (into the registers the z hops just freed), before the axpy and store.
// The arithmetic and its order are those of variant 6.  Only the plane ahead is
// held in registers: a thread's colour vectors of the current plane and of the
// plane behind are its own slots of the two LDS buffers (the plane ahead is
// written to the other buffer once the z hops have read the plane behind from
// it), which frees the registers and the copies of a three-plane ring.  On rows
// of 64 sites a wave is one row, and the backward x two-link is taken from the
// neighbouring lane instead of loaded.  With a one-link field (hops of one site)
// the tile marches consecutive planes and the LDS neighbours sit one row or
// column away (the two halo rows cover them).
template <int P, int R, bool NT>
__global__ __launch_bounds__(512) void step_zpipe(const StepGroup* __restrict__ groups, int n_groups,
                                                  int tile_base, int n_tiles, int tz, int rev,
                                                  const char* __restrict__ in, char* __restrict__ out,
                                                  typename Fmt<P>::real alpha, typename Fmt<P>::real beta) {
  using PL = Planes<P>;
  using real = typename Fmt<P>::real;
  using c2 = typename Complex2<real>::type;
  constexpr int D = hop_of(P);   // hop distance: 2 (two-links), 1 (one-links: one chain of consecutive planes)
  extern __shared__ __align__(16) unsigned char lds_raw[];
  c2* const lds = reinterpret_cast<c2*>(lds_raw);
  const TileSweep sw = xcd_sweep(n_tiles, rev);
  int it = 0;
  for (int m = 0; m < sw.n; m++) {
    const int tl = sw.tile(m);
    const int tile = tile_base + tl;
    const StepGroup& g = groups[find_group(groups, n_groups, tile)];
    const int Lx = g.Lx, Ly = g.Ly, Lz = g.Lz, rows = g.rows;
    const int64_t Vp = g.Vp;
    const int local = tile - g.tile_begin;
    const int tzi = local / g.n_xy_tiles;          // chain chunk index: n_z_tiles = chains * chunks
    const int y0 = (local - tzi * g.n_xy_tiles) * rows;
    const int chains = (D == 2 && !(Lz & 1)) ? 2 : 1;
    const int clen = Lz / chains;                  // planes per chain
    const int chunks = (clen + tz - 1) / tz;
    const int chain = tzi / chunks, chunk = tzi - chain * chunks;
    const int LxLy = Lx * Ly;
    const int t = (int)threadIdx.x;
    const int trow = t / Lx, x = t - trow * Lx;
    const bool active = trow < rows;
    // rows of 64 sites: a wave is one row and lane x holds W_x at x, so the backward x
    // two-link W_x(x - D) is lane x - D's forward one, taken across lanes instead of loaded
    const bool xlane = lane_xbw(P) && Lx == 64;
    const int row = active ? trow : 0;
    const int y = y0 + row;
    const int xy = y * Lx + x;
    const int xbw = y * Lx + wrap_sel(x - D, Lx);
    const int ybw = wrap_sel(y - D, Ly) * Lx + x;
    const int nsite = (rows + 4) * Lx;
    const int own = (row + 2) * Lx + x;
    const int sxf = (row + 2) * Lx + wrap_sel(x + D, Lx), sxb = (row + 2) * Lx + wrap_sel(x - D, Lx);
    const int syf = (row + 2 + D) * Lx + x, syb = (row + 2 - D) * Lx + x;
    const bool halo = t < 4 * Lx;
    const int hr = halo ? trow : 0;
    const int hrho = hr < 2 ? hr - 2 : rows + hr - 2;
    const int hxy = wrap_sel(y0 + hrho, Ly) * Lx + x;
    const int hslot = (hrho + 2) * Lx + x;
    const char* wp[3][PL::NW];
#pragma unroll
    for (int mu = 0; mu < 3; mu++) PL::w(g.W + mu * g.w_mu_stride, Vp, wp[mu]);
    const int nr = g.nr;
    const char* ip[R][PL::NV];
    char* op[R][PL::NV];
#pragma unroll
    for (int r = 0; r < R; r++) {
      const int64_t o = g.psi_off + (int64_t)min(r, nr - 1) * g.rhs_stride;
      PL::v(in + o, Vp, ip[r]);
      PL::v(out + o, Vp, op[r]);
    }
    const int k0 = chunk * tz;
    const int nz = min(k0 + tz, clen) - k0;        // planes of this chunk
    const bool up = ((chunk & 1) == 0) != (rev != 0);
    const int kf = up ? k0 : k0 + nz - 1;
    int z = wrap_sel(chain + D * kf, Lz);
    const int step = up ? D : -D;
    // ahd: colour vectors of the plane ahead in the march.  The current plane sits in
    // the thread's own slots of LDS buffer it & 1, the plane behind in those of the
    // other buffer.  wz[1]: the z link loaded for the current plane (W_z(z) marching
    // up, W_z(z-D) marching down), wz[0]: the one loaded for the previous plane.
    real ahd[R][6];
    real wz[2][18];
    real mxf[18], mxb[18], myf[18], myb[18];
    real hv[R][6];
    // a workgroup with several tiles: every thread has finished reading the previous
    // tile's LDS before the own slots of both buffers are written
    __syncthreads();
    {
      const uint32_t zo = (uint32_t)(z * LxLy);
      const uint32_t zc = zo + xy;
      real bh[R][6], cu[R][6];
#pragma unroll
      for (int r = 0; r < R; r++) {
        PL::load_v(ip[r], (uint32_t)(wrap_sel(z - step, Lz) * LxLy + xy), bh[r]);
        PL::load_v(ip[r], zc, cu[r]);
        PL::load_v(ip[r], (uint32_t)(wrap_sel(z + step, Lz) * LxLy + xy), ahd[r]);
        PL::load_v(ip[r], zo + hxy, hv[r]);
      }
      const uint32_t zm = (uint32_t)(wrap_sel(z - D, Lz) * LxLy + xy);
      PL::load_w(wp[2], up ? zm : zc, wz[0]);
      PL::load_w(wp[2], up ? zc : zm, wz[1]);
      PL::load_w_raw(wp[0], zc, mxf);
      if (!xlane) PL::load_w_raw(wp[0], zo + (uint32_t)xbw, mxb);
      PL::load_w_raw(wp[1], zc, myf);
      PL::load_w_raw(wp[1], zo + (uint32_t)ybw, myb);
      if (active) {
        c2* const bc = lds + (it & 1) * (R * 3) * nsite;
        c2* const bb = lds + ((it + 1) & 1) * (R * 3) * nsite;
#pragma unroll
        for (int r = 0; r < R; r++)
#pragma unroll
          for (int c = 0; c < 3; c++) {
            bb[(r * 3 + c) * nsite + own] = c2{bh[r][2 * c], bh[r][2 * c + 1]};
            bc[(r * 3 + c) * nsite + own] = c2{cu[r][2 * c], cu[r][2 * c + 1]};
          }
      }
    }
    // one plane step; MORE: a further plane follows in this chunk (the last step is
    // peeled off, so the loads for a next plane are unconditional inside the loop and
    // the registers they overwrite are not kept alive)
    auto plane_step = [&](auto more_c) {
      constexpr bool MORE = decltype(more_c)::value;
      const uint32_t site = (uint32_t)(z * LxLy) + xy;
      const int zn = wrap_sel(z + step, Lz);        // next plane of the march
      const uint32_t zno = (uint32_t)(zn * LxLy);
      c2* const buf = lds + (it & 1) * (R * 3) * nsite;           // current plane
      c2* const oth = lds + ((it + 1) & 1) * (R * 3) * nsite;     // own slots: the plane behind
      if (halo) {
#pragma unroll
        for (int r = 0; r < R; r++)
#pragma unroll
          for (int c = 0; c < 3; c++) buf[(r * 3 + c) * nsite + hslot] = c2{hv[r][2 * c], hv[r][2 * c + 1]};
      }
      // next plane: halo rows (the registers were just written to LDS); only the halo
      // threads load them (whole waves when the rows are 64 sites long)
      if constexpr (MORE) {
        if (halo) {
#pragma unroll
          for (int r = 0; r < R; r++) PL::load_v(ip[r], zno + (uint32_t)hxy, hv[r]);
        }
      }
      __syncthreads();
      if (xlane) {   // every lane of the wave is active here
        const int src = ((x - D) & 63) * 4;
#pragma unroll
        for (int c = 0; c < raw_words(P); c++) mxb[c] = lane_get(mxf[c], src);
      }
      PL::finish_w(mxf);
      PL::finish_w(mxb);
      PL::finish_w(myf);
      PL::finish_w(myb);
      // x hops of every RHS, then the y hops: per RHS the order (x fwd, x bwd, y fwd,
      // y bwd) is unchanged, and the next plane's x two-links can be issued in between
      real acc[R][6];
#pragma unroll
      for (int r = 0; r < R; r++) {
#pragma unroll
        for (int c = 0; c < 6; c++) acc[r][c] = (real)0;
        real v[6];
#pragma unroll
        for (int c = 0; c < 3; c++) { const c2 w = buf[(r * 3 + c) * nsite + sxf]; v[2 * c] = w.x; v[2 * c + 1] = w.y; }
        mv_acc(mxf, v, acc[r]);
#pragma unroll
        for (int c = 0; c < 3; c++) { const c2 w = buf[(r * 3 + c) * nsite + sxb]; v[2 * c] = w.x; v[2 * c + 1] = w.y; }
        mdv_acc(mxb, v, acc[r]);
      }
      // keep the next plane's loads below the hops that free their registers
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (MORE) {   // next plane: x two-links
        PL::load_w_raw(wp[0], zno + (uint32_t)xy, mxf);
        if (!xlane) PL::load_w_raw(wp[0], zno + (uint32_t)xbw, mxb);
      }
#pragma unroll
      for (int r = 0; r < R; r++) {
        real v[6];
#pragma unroll
        for (int c = 0; c < 3; c++) { const c2 w = buf[(r * 3 + c) * nsite + syf]; v[2 * c] = w.x; v[2 * c + 1] = w.y; }
        mv_acc(myf, v, acc[r]);
#pragma unroll
        for (int c = 0; c < 3; c++) { const c2 w = buf[(r * 3 + c) * nsite + syb]; v[2 * c] = w.x; v[2 * c + 1] = w.y; }
        mdv_acc(myb, v, acc[r]);
      }
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (MORE) {   // next plane: y two-links
        PL::load_w_raw(wp[1], zno + (uint32_t)xy, myf);
        PL::load_w_raw(wp[1], zno + (uint32_t)ybw, myb);
      }
      // z forward: W_z(z) psi(z+2); z backward: W_z(z-2)^dag psi(z-2)
      real bh[R][6];
#pragma unroll
      for (int r = 0; r < R; r++)
#pragma unroll
        for (int c = 0; c < 3; c++) { const c2 w = oth[(r * 3 + c) * nsite + own]; bh[r][2 * c] = w.x; bh[r][2 * c + 1] = w.y; }
      if (up) {
#pragma unroll
        for (int r = 0; r < R; r++) {
          mv_acc(wz[1], ahd[r], acc[r]);
          mdv_acc(wz[0], bh[r], acc[r]);
        }
      } else {
#pragma unroll
        for (int r = 0; r < R; r++) {
          mv_acc(wz[0], bh[r], acc[r]);
          mdv_acc(wz[1], ahd[r], acc[r]);
        }
      }
      // next plane: the plane ahead becomes its current plane (own slots of the other
      // buffer, after the plane behind was read from them); issue the colour vectors
      // ahead of the next plane and its z two-link before the axpy and store
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (MORE) {
        if (active) {
#pragma unroll
          for (int r = 0; r < R; r++)
#pragma unroll
            for (int c = 0; c < 3; c++) oth[(r * 3 + c) * nsite + own] = c2{ahd[r][2 * c], ahd[r][2 * c + 1]};
        }
#pragma unroll
        for (int c = 0; c < 18; c++) wz[0][c] = wz[1][c];
        const int za = wrap_sel(zn + step, Lz);
#pragma unroll
        for (int r = 0; r < R; r++) PL::load_v(ip[r], (uint32_t)(za * LxLy + xy), ahd[r]);
        PL::load_w(wp[2], up ? zno + (uint32_t)xy : (uint32_t)(wrap_sel(zn - D, Lz) * LxLy + xy), wz[1]);
      }
#pragma unroll
      for (int r = 0; r < R; r++) {
        real o[6];
#pragma unroll
        for (int c = 0; c < 3; c++) {
          const c2 w = buf[(r * 3 + c) * nsite + own];
          o[2 * c] = fma_(beta, acc[r][2 * c], alpha * w.x);
          o[2 * c + 1] = fma_(beta, acc[r][2 * c + 1], alpha * w.y);
        }
        if (active && r < nr) PL::template store_v<real, NT>(op[r], site, o);
      }
      z = zn;
      it++;
    };
    for (int i = 0; i + 1 < nz; i++) plane_step(std::true_type{});
    plane_step(std::false_type{});
  }
}

// Colour vectors of one plane of R RHS in LDS, rn = R * slots entries: FP32 as a 16-byte word
// (colours 0 and 1) and an 8-byte word (colour 2) per entry, each kind in its own array, so a
// vector is one 128-bit and one 64-bit LDS access; FP64 as three arrays of 16-byte words.
// With one RHS per group the compiler merges the two directions' z hops of the two-step
// kernel into one body that picks its link and vector arrays by address, which moves those
// register arrays to scratch memory.  An empty asm statement that differs between the two
// branches keeps them apart (one RHS only: with more, the merged form picks values in
// registers and costs nothing).
template <int R, int K>
__device__ __forceinline__ void keep_branch() {
  if constexpr (R == 1) {
    if constexpr (K == 0) asm volatile("; z hops of step one, upward march");
    else if constexpr (K == 1) asm volatile("; z hops of step one, downward march");
    else if constexpr (K == 2) asm volatile("; z hops of step two, upward march");
    else asm volatile("; z hops of step two, downward march");
  }
}

template <typename real> struct LdsVec;
template <> struct LdsVec<float> {
  static __device__ __forceinline__ int bytes(int rn) { return 24 * ((rn + 1) & ~1); }   // 16-byte aligned halves
  static __device__ __forceinline__ void put(unsigned char* p, int rn, int i, const float (&v)[6]) {
    reinterpret_cast<v4f*>(p)[i] = v4f{v[0], v[1], v[2], v[3]};
    reinterpret_cast<v2f*>(p + 16 * ((rn + 1) & ~1))[i] = v2f{v[4], v[5]};
  }
  static __device__ __forceinline__ void get(const unsigned char* p, int rn, int i, float (&v)[6]) {
    const v4f a = reinterpret_cast<const v4f*>(p)[i];
    const v2f b = reinterpret_cast<const v2f*>(p + 16 * ((rn + 1) & ~1))[i];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y;
  }
};
template <> struct LdsVec<double> {
  static __device__ __forceinline__ int bytes(int rn) { return 48 * rn; }
  static __device__ __forceinline__ void put(unsigned char* p, int rn, int i, const double (&v)[6]) {
#pragma unroll
    for (int c = 0; c < 3; c++) reinterpret_cast<v2d*>(p + 16 * rn * c)[i] = v2d{v[2 * c], v[2 * c + 1]};
  }
  static __device__ __forceinline__ void get(const unsigned char* p, int rn, int i, double (&v)[6]) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
      const v2d a = reinterpret_cast<const v2d*>(p + 16 * rn * c)[i];
      v[2 * c] = a.x;
      v[2 * c + 1] = a.y;
    }
  }
};

// Variant 8: two smearing steps per launch (temporal blocking).  The second
// step's input, the first step's output, never leaves the workgroup: each
// step-one result is rounded to the storage format in registers, exactly as a
// store and a reload would round it, and kept in LDS, so the pair of steps
// reads the two-links and the input once from memory and writes only the
// second step's output.  The arithmetic of both steps is that of the one-step
// kernels, so the result is bit-identical to two launches of any of them.
//
// Hops of D = 2 sites decouple the lattice into chains: the rows y, y+2, ...
// (two chains for even Ly, one for odd) and the planes z, z+2, ... (likewise).
// A tile is k consecutive rows of one y chain (full x extent) and a chunk of
// consecutive positions of one z chain.  The first step runs on the tile's
// rows plus one chain row on each side, which the second step's y hops read;
// its input plane is staged in LDS with a further chain row on each side.
// The march along the z chain keeps, per thread, its own column: stage s
// computes step one at march position m = s - 1 (input planes m - 1, m, m + 1)
// and step two at position m - 1 (step-one planes m - 2, m - 1, m), so a chunk
// of nz positions runs nz + 2 stages.  Two LDS buffers hold the input planes
// m (with its outer rows) and m - 1 (own slots), two more the step-one plane
// m - 1 and, in the thread's own slots, m - 2 (then m).  The z two-links
// between positions m - 2 .. m + 1 and step one's x two-links stay in
// registers for step two; its y two-links are reloaded.  One barrier per stage.  With one-link fields (D = 1) the chains are all rows and
// all planes.  XL: every group's rows are 64 sites long (a wave is one row, and the
// backward x two-link comes from the lane D to the left), fixed at compile time so
// that no register is set aside for loading it.
template <int P, int R, bool NT, bool XL>
__global__ __launch_bounds__(512) void step_fuse2(const StepGroup* __restrict__ groups, int n_groups,
                                                  int tile_base, int n_tiles, int tz, int rev,
                                                  const char* __restrict__ in, char* __restrict__ out,
                                                  typename Fmt<P>::real alpha, typename Fmt<P>::real beta) {
  using PL = Planes<P>;
  using real = typename Fmt<P>::real;
  using LV = LdsVec<real>;
  constexpr int D = hop_of(P);
  constexpr bool xlane = XL && lane_xbw(P);
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const TileSweep sw = xcd_sweep(n_tiles, rev);
  for (int mt = 0; mt < sw.n; mt++) {
    const int tile = tile_base + sw.tile(mt);
    const StepGroup& g = groups[find_group(groups, n_groups, tile)];
    const int Lx = XL ? 64 : g.Lx, Ly = g.Ly, Lz = g.Lz, k = g.rows;   // XL: every row is 64 sites long
    const int64_t Vp = g.Vp;
    const int local = tile - g.tile_begin;
    const int tzi = local / g.n_xy_tiles;          // z chain chunk index: n_z_tiles = chains * chunks
    const int yt = local - tzi * g.n_xy_tiles;     // y chain block index: n_xy_tiles = chains * blocks
    const int ychains = (D == 2 && !(Ly & 1)) ? 2 : 1;
    const int ylen = Ly / ychains;
    const int yblocks = ylen / k;
    const int ych = yt / yblocks, yb = yt - ych * yblocks;
    const int zchains = (D == 2 && !(Lz & 1)) ? 2 : 1;
    const int zlen = Lz / zchains;
    const int chunks = (zlen + tz - 1) / tz;
    const int zch = tzi / chunks, chunk = tzi - zch * chunks;
    const int LxLy = Lx * Ly;
    const int t = (int)threadIdx.x;
    const int trow = t / Lx, x = t - trow * Lx;
    // thread rows 0 .. k+1 are the chain rows -1 .. k of the block: step one on all of them,
    // step two on rows 1 .. k
    const bool inreg = trow < k + 2;
    const int row = inreg ? trow : 0;
    const bool core = inreg && row >= 1 && row <= k;
    auto lat_row = [&](int rel) { return wrap_sel(ych + D * wrap_sel(yb * k + rel, ylen), Ly); };
    const int y = lat_row(row - 1);
    const int xy = y * Lx + x;
    const int xbw = y * Lx + wrap_sel(x - D, Lx);
    const int ybw = lat_row(row - 2) * Lx + x;
    // LDS: input planes (k + 4 rows: chain rows -2 .. k+1), step-one planes (k + 2 rows)
    const int nA = (k + 4) * Lx, nB = (k + 2) * Lx;
    const int rnA = R * nA, rnB = R * nB;
    unsigned char* const A0 = lds_raw;
    unsigned char* const A1 = A0 + LV::bytes(rnA);
    unsigned char* const B0 = A1 + LV::bytes(rnA);
    unsigned char* const B1 = B0 + LV::bytes(rnB);
    const int xf = wrap_sel(x + D, Lx), xb = wrap_sel(x - D, Lx);
    const int oA = (row + 1) * Lx + x, aXf = (row + 1) * Lx + xf, aXb = (row + 1) * Lx + xb;
    const int aYf = (row + 2) * Lx + x, aYb = row * Lx + x;
    const int oB = row * Lx + x, bXf = row * Lx + xf, bXb = row * Lx + xb;
    const int bYf = (row + 1) * Lx + x, bYb = (row - 1) * Lx + x;   // read by core rows only
    // the input plane's outer rows (chain rows -2 and k+1) are loaded by the threads of rows
    // 0 and k+1, which have no step-two site, while the others run step two
    const bool edge = inreg && !core;
    const int hxy = lat_row(row == 0 ? -2 : k + 1) * Lx + x;
    const int hslot = (row == 0 ? 0 : k + 3) * Lx + x;
    const char* wp[3][PL::NW];
#pragma unroll
    for (int mu = 0; mu < 3; mu++) PL::w(g.W + mu * g.w_mu_stride, Vp, wp[mu]);
    const int nr = g.nr;
    const char* ip[R][PL::NV];
    char* op[R][PL::NV];
#pragma unroll
    for (int r = 0; r < R; r++) {
      const int64_t o = g.psi_off + (int64_t)min(r, nr - 1) * g.rhs_stride;
      PL::v(in + o, Vp, ip[r]);
      PL::v(out + o, Vp, op[r]);
    }
    const int k0 = chunk * tz;
    const int nz = min(k0 + tz, zlen) - k0;        // step-two positions of this chunk
    const bool up = ((chunk & 1) == 0) != (rev != 0);
    const int kf = up ? k0 : k0 + nz - 1;
    const int step = up ? D : -D;
    const int zf = wrap_step(zch + D * kf, 0, Lz);   // march position 0
    int zc = wrap_step(zf, -step, Lz);                // march position -1: step one's first plane
    const int zbb = wrap_step(zf, -2 * step, Lz);     // march position -2
    // z link between march positions a and a + 1: W_z at the lower of their planes
    auto link_site = [&](int za, int za1) { return (uint32_t)((up ? za : za1) * LxLy + xy); };
    real ahd[R][6];          // input colour vectors at march position m + 1 (own column)
    real lk[2][18];          // z links (m-1, m) and (m, m+1)
    real l0[18];             // z link (m-2, m-1)
    // x two-links: mxf of plane m (step one), mxp of plane m - 1 (step two), which step one's
    // mxf becomes once both are past their x hops, before the next plane's are loaded into
    // mxf; mxb, mbp: the backward ones (loaded when rows are not 64 sites long, else taken
    // from the neighbouring lane)
    real mxf[18], mxb[18], mxp[18], mbp[18];
    real myf[18], myb[18];
    // a workgroup with several tiles: every thread has finished reading the previous
    // tile's LDS before its own slots are written
    __syncthreads();
    {
      real bh[R][6], cu[R][6], hv[R][6];
#pragma unroll
      for (int r = 0; r < R; r++) {
        PL::load_v(ip[r], (uint32_t)(zbb * LxLy + xy), bh[r]);
        PL::load_v(ip[r], (uint32_t)(zc * LxLy + xy), cu[r]);
        PL::load_v(ip[r], (uint32_t)(zf * LxLy + xy), ahd[r]);
        PL::load_v(ip[r], (uint32_t)(zc * LxLy + hxy), hv[r]);
      }
      PL::load_w(wp[2], link_site(zbb, zc), lk[0]);
      PL::load_w(wp[2], link_site(zc, zf), lk[1]);
      const uint32_t zo = (uint32_t)(zc * LxLy);
      PL::load_w_raw(wp[0], zo + (uint32_t)xy, mxf);
      if (!xlane) PL::load_w_raw(wp[0], zo + (uint32_t)xbw, mxb);
      PL::load_w_raw(wp[1], zo + (uint32_t)xy, myf);
      PL::load_w_raw(wp[1], zo + (uint32_t)ybw, myb);
      if (inreg) {
#pragma unroll
        for (int r = 0; r < R; r++)
          {
            LV::put(A0, rnA, r * nA + oA, cu[r]);
            LV::put(A1, rnA, r * nA + oA, bh[r]);
          }
      }
      if (edge) {
#pragma unroll
        for (int r = 0; r < R; r++)
          LV::put(A0, rnA, r * nA + hslot, hv[r]);
      }
    }
    int s = 0;
    // one stage; S2: step two runs (s >= 2); MORE: a further stage follows
    auto stage = [&](auto s2_c, auto more_c) {
      constexpr bool S2 = decltype(s2_c)::value;
      constexpr bool MORE = decltype(more_c)::value;
      // step one's x two-links become step two's, and the next plane's are loaded
      auto next_x = [&]() {
#pragma unroll
        for (int c = 0; c < 18; c++) mxp[c] = mxf[c];
        if (!xlane) {
#pragma unroll
          for (int c = 0; c < 18; c++) mbp[c] = mxb[c];
        }
        const uint32_t zno = (uint32_t)(wrap_sel(zc + step, Lz) * LxLy);
        PL::load_w_raw(wp[0], zno + (uint32_t)xy, mxf);
        if (!xlane) PL::load_w_raw(wp[0], zno + (uint32_t)xbw, mxb);
      };
      const int zn = wrap_sel(zc + step, Lz);   // march position m + 1
      const int zb = wrap_sel(zc - step, Lz);   // march position m - 1
      unsigned char* const Ac = (s & 1) ? A1 : A0;          // input plane m; own slots of Ao: plane m - 1
      unsigned char* const Ao = (s & 1) ? A0 : A1;          // (then plane m + 1, with its outer rows)
      unsigned char* const Bc = (s & 1) ? B1 : B0;          // own slots: step one at m - 2, then at m
      unsigned char* const Bo = (s & 1) ? B0 : B1;          // step one at m - 1
      __syncthreads();
      // ---- step one at plane zc, chain rows -1 .. k
      if (xlane) {
        const int src = ((x - D) & 63) * 4;
#pragma unroll
        for (int c = 0; c < raw_words(P); c++) mxb[c] = lane_get(mxf[c], src);
      }
      PL::finish_w(mxf);
      PL::finish_w(mxb);
      PL::finish_w(myf);
      PL::finish_w(myb);
      real acc[R][6];
#pragma unroll
      for (int r = 0; r < R; r++) {
#pragma unroll
        for (int c = 0; c < 6; c++) acc[r][c] = (real)0;
        real v[6];
        LV::get(Ac, rnA, r * nA + aXf, v);
        mv_acc(mxf, v, acc[r]);
        LV::get(Ac, rnA, r * nA + aXb, v);
        mdv_acc(mxb, v, acc[r]);
      }
#pragma unroll
      for (int r = 0; r < R; r++) {
        real v[6];
        LV::get(Ac, rnA, r * nA + aYf, v);
        mv_acc(myf, v, acc[r]);
        LV::get(Ac, rnA, r * nA + aYb, v);
        mdv_acc(myb, v, acc[r]);
      }
      __builtin_amdgcn_sched_barrier(0);
      // the next plane's x two-links now when no step two runs, else after its x hops; the
      // y two-links of the next use (step two at plane zb, else step one at plane zn) now
      const uint32_t zno = (uint32_t)(zn * LxLy);
      const uint32_t zon = (uint32_t)((S2 ? zb : zn) * LxLy);
      if constexpr (MORE && !S2) next_x();
      if constexpr (S2 || MORE) {
        PL::load_w_raw(wp[1], zon + (uint32_t)xy, myf);
        PL::load_w_raw(wp[1], zon + (uint32_t)ybw, myb);
      }
      {
        real bh[R][6];
#pragma unroll
        for (int r = 0; r < R; r++)
          LV::get(Ao, rnA, r * nA + oA, bh[r]);
        if (up) {
#pragma unroll
          for (int r = 0; r < R; r++) {
            mv_acc(lk[1], ahd[r], acc[r]);
            mdv_acc(lk[0], bh[r], acc[r]);
          }
          keep_branch<R, 0>();
        } else {
#pragma unroll
          for (int r = 0; r < R; r++) {
            mv_acc(lk[0], bh[r], acc[r]);
            mdv_acc(lk[1], ahd[r], acc[r]);
          }
          keep_branch<R, 1>();
        }
      }
      real s1[R][6];
#pragma unroll
      for (int r = 0; r < R; r++) {
        real w[6];
        LV::get(Ac, rnA, r * nA + oA, w);
#pragma unroll
        for (int c = 0; c < 6; c++) s1[r][c] = fma_(beta, acc[r][c], alpha * w[c]);
        PL::round_v(s1[r]);
      }
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (MORE) {   // input plane m + 1 becomes the next stage's current plane
        if (inreg) {
#pragma unroll
          for (int r = 0; r < R; r++)
            LV::put(Ao, rnA, r * nA + oA, ahd[r]);
        }
        const int znn = wrap_sel(zn + step, Lz);   // the next stage's input plane ahead
#pragma unroll
        for (int r = 0; r < R; r++) PL::load_v(ip[r], (uint32_t)(znn * LxLy + xy), ahd[r]);
      }
      // ---- step two at plane zb, chain rows 0 .. k-1; meanwhile the edge rows load the outer
      // rows of input plane m + 1 into Ao (whose outer rows were last read before this
      // stage's barrier)
      if constexpr (MORE) {
        if (edge) {
          real hv[R][6];
#pragma unroll
          for (int r = 0; r < R; r++) PL::load_v(ip[r], (uint32_t)(zn * LxLy + hxy), hv[r]);
#pragma unroll
          for (int r = 0; r < R; r++)
            LV::put(Ao, rnA, r * nA + hslot, hv[r]);
        }
      }
      if constexpr (S2) {
        if (core) {   // mxp was completed by step one at the previous stage
          if (xlane) {
            const int src = ((x - D) & 63) * 4;
#pragma unroll
            for (int c = 0; c < 18; c++) mbp[c] = lane_get(mxp[c], src);
          }
#pragma unroll
          for (int r = 0; r < R; r++) {
#pragma unroll
            for (int c = 0; c < 6; c++) acc[r][c] = (real)0;
            real v[6];
            LV::get(Bo, rnB, r * nB + bXf, v);
            mv_acc(mxp, v, acc[r]);
            LV::get(Bo, rnB, r * nB + bXb, v);
            mdv_acc(mbp, v, acc[r]);
          }
        }
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (MORE) next_x();
        if (core) {
          PL::finish_w(myf);
          PL::finish_w(myb);
#pragma unroll
          for (int r = 0; r < R; r++) {
            real v[6];
            LV::get(Bo, rnB, r * nB + bYf, v);
            mv_acc(myf, v, acc[r]);
            LV::get(Bo, rnB, r * nB + bYb, v);
            mdv_acc(myb, v, acc[r]);
          }
        }
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (MORE) {
          PL::load_w_raw(wp[1], zno + (uint32_t)xy, myf);
          PL::load_w_raw(wp[1], zno + (uint32_t)ybw, myb);
        }
        if (core) {
          real bh[R][6];
#pragma unroll
          for (int r = 0; r < R; r++)
            LV::get(Bc, rnB, r * nB + oB, bh[r]);
          if (up) {
#pragma unroll
            for (int r = 0; r < R; r++) {
              mv_acc(lk[0], s1[r], acc[r]);
              mdv_acc(l0, bh[r], acc[r]);
            }
            keep_branch<R, 2>();
          } else {
#pragma unroll
            for (int r = 0; r < R; r++) {
              mv_acc(l0, bh[r], acc[r]);
              mdv_acc(lk[0], s1[r], acc[r]);
            }
            keep_branch<R, 3>();
          }
          const uint32_t site = (uint32_t)(zb * LxLy + xy);
#pragma unroll
          for (int r = 0; r < R; r++) {
            real o[6];
            real w[6];
            LV::get(Bo, rnB, r * nB + oB, w);
#pragma unroll
            for (int c = 0; c < 6; c++) o[c] = fma_(beta, acc[r][c], alpha * w[c]);
            if (r < nr) PL::template store_v<real, NT>(op[r], site, o);
          }
        }
      }
      if (inreg) {   // step one at m: the own slots of Bc (step one at m - 2 is no longer read)
#pragma unroll
        for (int r = 0; r < R; r++)
          LV::put(Bc, rnB, r * nB + oB, s1[r]);
      }
#pragma unroll
      for (int c = 0; c < 18; c++) {
        l0[c] = lk[0][c];
        lk[0][c] = lk[1][c];
      }
      if constexpr (MORE) {   // the next stage's z link
        PL::load_w(wp[2], link_site(zn, wrap_sel(zn + step, Lz)), lk[1]);
      }
      zc = zn;
      s++;
    };
    stage(std::false_type{}, std::true_type{});   // step one at march position -1
    stage(std::false_type{}, std::true_type{});   // step one at 0
    for (int i = 1; i < nz; i++) stage(std::true_type{}, std::true_type{});
    stage(std::true_type{}, std::false_type{});   // step one at nz, step two at nz - 1
  }
}

constexpr int kMaxLds = 160 * 1024;   // LDS per compute unit on gfx950

// Variant 8, with rows of 64 sites fixed at compile time where the form uses the lane exchange.
template <int P, int R, bool NT>
hipError_t launch_fuse2(const StepConfig& cfg, int grid, const StepGroup* groups, int n_groups, int tile_base,
                        int n_tiles, const char* in, char* out, typename Fmt<P>::real a, typename Fmt<P>::real b,
                        int64_t lds, hipStream_t s) {
  if constexpr (lane_xbw(P)) {
    if (cfg.rows64) {
      step_fuse2<P, R, NT, true><<<grid, cfg.block, (size_t)lds, s>>>(groups, n_groups, tile_base, n_tiles, cfg.tz,
                                                                       cfg.rev, in, out, a, b);
      return hipGetLastError();
    }
  }
  step_fuse2<P, R, NT, false><<<grid, cfg.block, (size_t)lds, s>>>(groups, n_groups, tile_base, n_tiles, cfg.tz, cfg.rev,
                                                                    in, out, a, b);
  return hipGetLastError();
}

template <int P, int R, bool NT>
hipError_t launch_step_n(const StepConfig& cfg, const StepGroup* groups, int n_groups, int tile_base,
                         int n_tiles, const char* in, char* out, double alpha, double beta, int64_t lds,
                         hipStream_t s) {
  using real = typename Fmt<P>::real;
  const int grid = cfg.grid > 0 ? std::min(cfg.grid, n_tiles) : n_tiles;
  // The ring kernels are instantiated only where their registers fit; FP64 with wider
  // groups runs the direct kernel, which computes the same bits.
  // (variant 5 has full-row tiles and its own block sizes: it never falls back, and the host
  // never selects it for FP64 groups wider than one RHS)
  if (cfg.variant >= 5 && vprec(P) == F64 && R > 1) return hipErrorInvalidValue;
  if constexpr (is_one(P)) {   // one-link fields: hops of one site, variants 0, 4, 7 and 8
    const real a = (real)alpha, b = (real)beta;
    if (cfg.variant == 0)
      step_direct<P, R, NT><<<grid, cfg.block, 0, s>>>(groups, n_groups, tile_base, n_tiles, cfg.tz, cfg.rev, in, out, a, b);
    else if (cfg.variant == 4)
      step_rolled<P, R, NT><<<grid, cfg.block, 0, s>>>(groups, n_groups, tile_base, n_tiles, cfg.tz, cfg.rev, in, out, a, b);
    else if (cfg.variant == 7 || cfg.variant == 8) {
      constexpr int R2 = (vprec(P) == F64) ? 1 : R;
      if (lds <= 0 || lds > kMaxLds) return hipErrorInvalidValue;
      if (cfg.variant == 7)
        step_zpipe<P, R2, NT><<<grid, cfg.block, (size_t)lds, s>>>(groups, n_groups, tile_base, n_tiles, cfg.tz, cfg.rev,
                                                                  in, out, a, b);
      else
        return launch_fuse2<P, R2, NT>(cfg, grid, groups, n_groups, tile_base, n_tiles, in, out, a, b, lds, s);
    } else
      return hipErrorInvalidValue;
    return hipGetLastError();
  } else {   // two-link fields: every variant
    const bool direct = cfg.variant == 0 || (vprec(P) == F64 && R > (cfg.variant == 1 ? 2 : 1) && cfg.variant != 4 &&
                                             cfg.variant < 5);
    (void)lds;
    constexpr int R1 = (vprec(P) == F64 && R > 2) ? 1 : R;
    constexpr int R2 = (vprec(P) == F64) ? 1 : R;
    const real a = (real)alpha, b = (real)beta;
    if (direct)
      step_direct<P, R, NT><<<grid, cfg.block, 0, s>>>(groups, n_groups, tile_base, n_tiles, cfg.tz, cfg.rev, in, out, a, b);
    else if (cfg.variant == 1)
      step_zmarch<P, R1, NT><<<grid, cfg.block, 0, s>>>(groups, n_groups, tile_base, n_tiles, cfg.tz, cfg.rev, in, out, a, b);
    else if (cfg.variant == 2)
      step_zring<P, R2, NT><<<grid, cfg.block, 0, s>>>(groups, n_groups, tile_base, n_tiles, cfg.tz, cfg.rev, in, out, a, b);
    else if (cfg.variant == 3)
      step_zfront<P, R2, NT><<<grid, cfg.block, 0, s>>>(groups, n_groups, tile_base, n_tiles, cfg.tz, cfg.rev, in, out, a, b);
    else if (cfg.variant == 4)
      step_rolled<P, R, NT><<<grid, cfg.block, 0, s>>>(groups, n_groups, tile_base, n_tiles, cfg.tz, cfg.rev, in, out, a, b);
    else if (cfg.variant == 7) {
      if (lds <= 0 || lds > kMaxLds) return hipErrorInvalidValue;
      step_zpipe<P, R2, NT><<<grid, cfg.block, (size_t)lds, s>>>(groups, n_groups, tile_base, n_tiles, cfg.tz, cfg.rev, in, out,
                                                                a, b);
    } else if (cfg.variant == 8) {
      if (lds <= 0 || lds > kMaxLds) return hipErrorInvalidValue;
      return launch_fuse2<P, R2, NT>(cfg, grid, groups, n_groups, tile_base, n_tiles, in, out, a, b, lds, s);
    } else if (cfg.variant == 6) {
      if (lds <= 0 || lds > kMaxLds) return hipErrorInvalidValue;
      step_zchain<P, R2, NT><<<grid, cfg.block, (size_t)lds, s>>>(groups, n_groups, tile_base, n_tiles, cfg.tz, cfg.rev, in, out,
                                                                 a, b);
    } else if (cfg.variant == 5) {
      if (lds <= 0 || lds > kMaxLds) return hipErrorInvalidValue;
      step_zlds<P, R2, NT><<<grid, cfg.block, (size_t)lds, s>>>(groups, n_groups, tile_base, n_tiles, cfg.tz, cfg.rev, in, out,
                                                               a, b);
    } else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
}

template <int P, int R>
hipError_t launch_step_t(const StepConfig& cfg, const StepGroup* groups, int n_groups, int tile_base,
                         int n_tiles, const char* in, char* out, double alpha, double beta, int64_t lds,
                         hipStream_t s) {
  if (cfg.nt)
    return launch_step_n<P, R, true>(cfg, groups, n_groups, tile_base, n_tiles, in, out, alpha, beta, lds, s);
  return launch_step_n<P, R, false>(cfg, groups, n_groups, tile_base, n_tiles, in, out, alpha, beta, lds, s);
}

template <int P, int R>
hipError_t allow_lds() {
  if constexpr (is_one(P)) {
    for (const void* f : {reinterpret_cast<const void*>(&step_zpipe<P, R, false>),
                          reinterpret_cast<const void*>(&step_zpipe<P, R, true>),
                          reinterpret_cast<const void*>(&step_fuse2<P, R, false, false>),
                          reinterpret_cast<const void*>(&step_fuse2<P, R, true, false>),
                          reinterpret_cast<const void*>(&step_fuse2<P, R, false, lane_xbw(P)>),
                          reinterpret_cast<const void*>(&step_fuse2<P, R, true, lane_xbw(P)>)}) {
      const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  } else {
    for (const void* f : {reinterpret_cast<const void*>(&step_zlds<P, R, false>),
                          reinterpret_cast<const void*>(&step_zlds<P, R, true>),
                          reinterpret_cast<const void*>(&step_zchain<P, R, false>),
                          reinterpret_cast<const void*>(&step_zchain<P, R, true>),
                          reinterpret_cast<const void*>(&step_zpipe<P, R, false>),
                          reinterpret_cast<const void*>(&step_zpipe<P, R, true>),
                          reinterpret_cast<const void*>(&step_fuse2<P, R, false, false>),
                          reinterpret_cast<const void*>(&step_fuse2<P, R, true, false>),
                          reinterpret_cast<const void*>(&step_fuse2<P, R, false, lane_xbw(P)>),
                          reinterpret_cast<const void*>(&step_fuse2<P, R, true, lane_xbw(P)>)}) {
      const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
}

template <int P>
hipError_t launch_step_p(int width, const StepConfig& cfg, const StepGroup* groups, int n_groups, int tile_base,
                         int n_tiles, const char* in, char* out, double alpha, double beta, int64_t lds,
                         hipStream_t s) {
  switch (width) {
    case 1: return launch_step_t<P, 1>(cfg, groups, n_groups, tile_base, n_tiles, in, out, alpha, beta, lds, s);
    case 2: return launch_step_t<P, 2>(cfg, groups, n_groups, tile_base, n_tiles, in, out, alpha, beta, lds, s);
    case 3: return launch_step_t<P, 3>(cfg, groups, n_groups, tile_base, n_tiles, in, out, alpha, beta, lds, s);
    case 4: return launch_step_t<P, 4>(cfg, groups, n_groups, tile_base, n_tiles, in, out, alpha, beta, lds, s);
    default: return hipErrorInvalidValue;
  }
}

// Every link form of storage precision P (form = code & (W12 | ONE)).
template <int P>
hipError_t launch_step_both(int form, int width, const StepConfig& cfg, const StepGroup* groups, int n_groups,
                            int tile_base, int n_tiles, const char* in, char* out, double alpha, double beta,
                            int64_t lds, hipStream_t s) {
  switch (form) {
    case 0: return launch_step_p<P>(width, cfg, groups, n_groups, tile_base, n_tiles, in, out, alpha, beta, lds, s);
    case W12: return launch_step_p<P | W12>(width, cfg, groups, n_groups, tile_base, n_tiles, in, out, alpha, beta, lds, s);
    case ONE: return launch_step_p<P | ONE>(width, cfg, groups, n_groups, tile_base, n_tiles, in, out, alpha, beta, lds, s);
    case W12 | ONE:
      return launch_step_p<P | W12 | ONE>(width, cfg, groups, n_groups, tile_base, n_tiles, in, out, alpha, beta, lds, s);
    default: return hipErrorInvalidValue;
  }
}

template <int P>
hipError_t step_attributes_both() {
  hipError_t e = hipSuccess;
  if constexpr (P == F64) {
    for (hipError_t r : {allow_lds<P, 1>(), allow_lds<P | W12, 1>(), allow_lds<P | ONE, 1>(),
                         allow_lds<P | W12 | ONE, 1>()})
      if (r != hipSuccess) e = r;
  } else {
    for (hipError_t r : {allow_lds<P, 1>(), allow_lds<P, 2>(), allow_lds<P, 3>(), allow_lds<P, 4>(),
                         allow_lds<P | W12, 1>(), allow_lds<P | W12, 2>(), allow_lds<P | W12, 3>(),
                         allow_lds<P | W12, 4>(), allow_lds<P | ONE, 1>(), allow_lds<P | ONE, 2>(),
                         allow_lds<P | ONE, 3>(), allow_lds<P | ONE, 4>(), allow_lds<P | W12 | ONE, 1>(),
                         allow_lds<P | W12 | ONE, 2>(), allow_lds<P | W12 | ONE, 3>(),
                         allow_lds<P | W12 | ONE, 4>()})
      if (r != hipSuccess) e = r;
  }
  return e;
}

}  // namespace

}  // namespace tl
