// HIP kernels for gfx950 other than the smearing step (tl_step.h): two-link
// build, pack/unpack, FP64 reductions, buffer comparison; the step dispatch.

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "tl_format.h"
#include "tl_internal.h"
#include "tl_step.h"

namespace tl {

namespace {

// ------------------------------------------------------------------ build

constexpr int kBuildSites = 21;                    // sites per chunk: 63 (site, mu) pairs, one per lane
constexpr int kBuildWaves = 4;                     // waves per workgroup
constexpr int kBuildWords = 9 * 3 * kBuildSites;   // 16-byte words of a chunk's 63 matrices
constexpr int kBuildLoads = (kBuildWords + 63) / 64;

// Coalesced loads of one chunk (kBuildSites consecutive sites s0.. of the slice at Ut):
// word w of the chunk's own matrices is word w % 27 of site w / 27 (its spatial links, the
// t link skipped); word w of the neighbour matrices is word w % 9 of the neighbour link
// U_mu(x + mu^) of pair p = w / 9 (site p / 3, mu = p % 3), whose site index lane p computes
// and shares by a shuffle.  Sites past the slice end read the last site.
template <bool ONE>
__device__ __forceinline__ void build_load(const v2d* __restrict__ Ut, int s0, int V3, int Lx, int Ly, int Lz,
                                           int lane, v2d (&va)[kBuildLoads], v2d (&vb)[kBuildLoads]) {
  const int lp = min(lane, 3 * kBuildSites - 1);
  const int ps = lp / 3, mu = lp - 3 * ps;
  const int ii = min(s0 + ps, V3 - 1);
  const int x = ii % Lx, yz = ii / Lx, y = yz % Ly, z = yz / Ly;
  const int xp = x + 1 == Lx ? 0 : x + 1, yp = y + 1 == Ly ? 0 : y + 1, zp = z + 1 == Lz ? 0 : z + 1;
  const int nbl = mu == 0 ? (z * Ly + y) * Lx + xp : mu == 1 ? (z * Ly + yp) * Lx + x : (zp * Ly + y) * Lx + x;
#pragma unroll
  for (int k = 0; k < kBuildLoads; k++) {
    const int w = min(lane + 64 * k, kBuildWords - 1);
    const int site = w / 27, q = w - 27 * site;
    va[k] = Ut[(int64_t)min(s0 + site, V3 - 1) * 36 + q];
    if constexpr (!ONE) {
      const int p = w / 9, jw = w - 9 * p;
      vb[k] = Ut[(int64_t)__shfl(nbl, p, 64) * 36 + (p - 3 * (p / 3)) * 9 + jw];
    }
  }
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// W_mu(x) = U_mu(x) U_mu(x + mu^) in FP64, stored in format P; with the ONE bit in P the
// links U_mu(x) themselves (a one-link field).  A chunk of 21 consecutive sites is one
// wave's work, one (site, mu) pair per lane, mu fastest.  A lane's own matrix and its
// neighbour's are 144-byte runs 576 bytes apart (the caller's layout interleaves the t
// links): lanes loading them directly would each touch their own cache lines, and the
// texture addresser rather than HBM would bound the kernel.  So the wave loads the chunk's
// words with consecutive lanes on consecutive words (build_load), writes them to its part
// of LDS, and each lane reads its two matrices back.  A workgroup takes four consecutive
// chunks of one slice.
template <int P>
__global__ __launch_bounds__(64 * kBuildWaves) void build_twolinks_kernel(const double2* __restrict__ U, int Lx, int Ly,
                                                                           int Lz, int t_first, int slot_first,
                                                                           int per_slice, char* __restrict__ W,
                                                                           int64_t Vp) {
  constexpr bool one = is_one(P);
  __shared__ v2d lds[kBuildWaves][2][kBuildLoads * 64];
  const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
  const int V3 = Lx * Ly * Lz;
  const int sl = (int)blockIdx.x / per_slice;
  const int s0 = (((int)blockIdx.x - sl * per_slice) * kBuildWaves + wave) * kBuildSites;
  if (s0 >= V3) return;   // wave-uniform: a slice's last workgroup may have idle waves
  v2d(&own)[kBuildLoads * 64] = lds[wave][0];
  v2d(&nbr)[kBuildLoads * 64] = lds[wave][1];
  {
    v2d va[kBuildLoads], vb[kBuildLoads];
    build_load<one>(reinterpret_cast<const v2d*>(U) + (int64_t)(t_first + sl) * V3 * 36, s0, V3, Lx, Ly, Lz, lane,
                    va, vb);
#pragma unroll
    for (int k = 0; k < kBuildLoads; k++) {
      own[lane + 64 * k] = va[k];
      if constexpr (!one) nbr[lane + 64 * k] = vb[k];
    }
  }
  wave_sync_lds();   // each lane reads words other lanes of its wave wrote
  const int lp = min(lane, 3 * kBuildSites - 1);
  const int ps = lp / 3, mu = lp - 3 * ps;
  if (lane >= 3 * kBuildSites || s0 + ps >= V3) return;
  v2d a[9];
#pragma unroll
  for (int q = 0; q < 9; q++) a[q] = own[9 * lp + q];
  double m[18];
  if constexpr (one) {
#pragma unroll
    for (int q = 0; q < 9; q++) {
      m[2 * q] = a[q].x;
      m[2 * q + 1] = a[q].y;
    }
  } else {
    v2d bq[9];
#pragma unroll
    for (int q = 0; q < 9; q++) bq[q] = nbr[9 * lp + q];
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
      for (int t = 0; t < 3; t++) {
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int q = 0; q < 3; q++) {
          const v2d pa = a[3 * r + q], pb = bq[3 * q + t];
          re = fma_(pa.x, pb.x, re);
          re = fma_(-pa.y, pb.y, re);
          im = fma_(pa.x, pb.y, im);
          im = fma_(pa.y, pb.x, im);
        }
        m[2 * (3 * r + t)] = re;
        m[2 * (3 * r + t) + 1] = im;
      }
  }
  char* const Wm = W + ((int64_t)(slot_first + sl) * 3 + mu) * Vp * kWBytes[P];
  Fmt<P>::store_w(Wm, Vp, s0 + ps, m);
}

// ------------------------------------------------------------------ pack / unpack

template <int P>
__global__ __launch_bounds__(256) void pack_kernel(const double2* __restrict__ nat, char* __restrict__ packed,
                                                   const int64_t* __restrict__ rhs_off, int64_t V3, int64_t Vp) {
  const int r = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V3) return;
  const double2* s = nat + ((int64_t)r * V3 + i) * 3;
  double v[6];
#pragma unroll
  for (int c = 0; c < 3; c++) {
    const double2 w = s[c];
    v[2 * c] = w.x;
    v[2 * c + 1] = w.y;
  }
  Fmt<P>::store_v(packed + rhs_off[r], Vp, i, v);
}

template <int P>
__global__ __launch_bounds__(256) void unpack_kernel(const char* __restrict__ packed, double2* __restrict__ nat,
                                                     const int64_t* __restrict__ rhs_off, int64_t V3, int64_t Vp) {
  const int r = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V3) return;
  double v[6];
  Fmt<P>::load_v(packed + rhs_off[r], Vp, i, v);
  double2* d = nat + ((int64_t)r * V3 + i) * 3;
#pragma unroll
  for (int c = 0; c < 3; c++) d[c] = make_double2(v[2 * c], v[2 * c + 1]);
}

// ------------------------------------------------------------------ reductions

constexpr int kRedBlock = 256;
constexpr int kRedSitesPerBlock = 4096;

// Natural complex128 vectors: [..][site][3].
struct NatLoad {
  __device__ static void load(const char* b, int64_t off, int64_t Vp, int64_t i, double (&v)[6]) {
    (void)Vp;
    const double2* p = reinterpret_cast<const double2*>(b) + off + i * 3;
#pragma unroll
    for (int c = 0; c < 3; c++) {
      const double2 w = p[c];
      v[2 * c] = w.x;
      v[2 * c + 1] = w.y;
    }
  }
};

template <int P>
struct PackedLoad {
  __device__ static void load(const char* b, int64_t off, int64_t Vp, int64_t i, double (&v)[6]) {
    Fmt<P>::load_v(b + off, Vp, i, v);
  }
};

__device__ __forceinline__ double block_sum(double v, double* lds) {
  // wave64 butterfly, then the waves' partial sums in wave order
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); w++) s += lds[w];
  __syncthreads();
  return s;
}

// Where the fields of a reduction lie: a device table with one entry per RHS, or natural
// fields of n sites each, one after the other (the entry is then computed, no table).
struct TableFields {
  const RedField* f;
  __device__ RedField operator()(int r) const { return f[r]; }
};
struct FlatFields {
  int64_t n;
  __device__ RedField operator()(int r) const {
    const int64_t o = (int64_t)r * n;
    return RedField{3 * o, 3 * o, n, 0, o};
  }
};

// partials[(r * nb + b) * 2 + {0,1}]: block b of RHS r.  Fixed site-to-block
// and in-block orders make the result reproducible run to run.
template <class LD, class F>
__global__ __launch_bounds__(kRedBlock) void reduce_partial_kernel(int kind, const char* __restrict__ a,
                                                                   const char* __restrict__ b, F f,
                                                                   double* __restrict__ partials) {
  __shared__ double lds[kRedBlock / 64];
  const int r = blockIdx.y;
  const int nb = gridDim.x;
  const RedField fr = f(r);
  const int64_t s0 = (int64_t)blockIdx.x * kRedSitesPerBlock;
  const int64_t s1 = min(s0 + (int64_t)kRedSitesPerBlock, fr.V3);
  double re = 0.0, im = 0.0;
  for (int64_t i = s0 + threadIdx.x; i < s1; i += blockDim.x) {
    double v[6];
    LD::load(a, fr.off, fr.Vp, i, v);
    if (kind == 0) {
#pragma unroll
      for (int c = 0; c < 6; c++) re = fma_(v[c], v[c], re);
    } else {
      double u[6];
      LD::load(b, fr.off2, fr.Vp, i, u);   // <u, v> = sum conj(u) v
#pragma unroll
      for (int c = 0; c < 3; c++) {
        re = fma_(u[2 * c], v[2 * c], re);
        re = fma_(u[2 * c + 1], v[2 * c + 1], re);
        im = fma_(u[2 * c], v[2 * c + 1], im);
        im = fma_(-u[2 * c + 1], v[2 * c], im);
      }
    }
  }
  re = block_sum(re, lds);
  if (kind == 1) im = block_sum(im, lds);
  if (threadIdx.x == 0) {
    partials[((int64_t)r * nb + blockIdx.x) * 2] = re;
    partials[((int64_t)r * nb + blockIdx.x) * 2 + 1] = im;
  }
}

__global__ void reduce_finish_kernel(int kind, const double* __restrict__ partials, int nb, int n_rhs,
                                     double* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_rhs) return;
  double re = 0.0, im = 0.0;
  for (int k = 0; k < nb; k++) {
    re += partials[((int64_t)r * nb + k) * 2];
    im += partials[((int64_t)r * nb + k) * 2 + 1];
  }
  if (kind == 0) {
    out[r] = re;
  } else {
    out[2 * r] = re;
    out[2 * r + 1] = im;
  }
}

template <class LD, class F>
__global__ __launch_bounds__(kRedBlock) void site_norm_kernel(const char* __restrict__ a, F f,
                                                              double* __restrict__ out) {
  const int r = blockIdx.y;
  const RedField fr = f(r);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= fr.V3) return;
  double v[6];
  LD::load(a, fr.off, fr.Vp, i, v);
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < 6; c++) s = fma_(v[c], v[c], s);
  out[fr.out_off + i] = sqrt(s);
}

// Streaming probe: out[i] = sum of the n_in input planes' word i (FP32 adds), n_in reads
// per write, loads cached or nontemporal (NTL), stores cached or nontemporal (NTS).  Each
// thread handles four words per pass of a grid-stride loop.
template <bool NTL, bool NTS>
__global__ __launch_bounds__(256) void stream_kernel(const v4f* __restrict__ in, int n_in, v4f* __restrict__ out,
                                                      int64_t n_words) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < n_words; i0 += 4 * stride) {
    v4f acc[4] = {};
    for (int p = 0; p < n_in; p++) {
      const v4f* src = in + (int64_t)p * n_words;
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const int64_t i = min(i0 + u * stride, n_words - 1);
        acc[u] += NTL ? __builtin_nontemporal_load(src + i) : src[i];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; u++)
      if (i0 + u * stride < n_words) put<NTS>(out + i0 + u * stride, acc[u]);
  }
}

__global__ void compare_kernel(const uint4* __restrict__ a, const uint4* __restrict__ b, int64_t n16,
                               const unsigned char* __restrict__ ta, const unsigned char* __restrict__ tb,
                               int64_t ntail, int* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool diff = false;
  for (int64_t k = i; k < n16; k += stride) {
    const uint4 x = a[k], y = b[k];
    diff |= (x.x != y.x) | (x.y != y.y) | (x.z != y.z) | (x.w != y.w);
  }
  for (int64_t k = i; k < ntail; k += stride) diff |= ta[k] != tb[k];
  if (diff) *flag = 1;
}


}  // namespace

hipError_t init_kernel_attributes() {
  hipError_t e = hipSuccess;
  for (hipError_t r : {step_attributes_f64(), step_attributes_f32(), step_attributes_f16s(), step_attributes_bf16()})
    if (r != hipSuccess) e = r;
  return e;
}

hipError_t launch_step(int code, int width, const StepConfig& cfg, const StepGroup* groups, int n_groups,
                       int tile_base, int n_tiles, const char* in, char* out, double alpha, double beta, int64_t lds,
                       hipStream_t stream) {
  if (n_tiles <= 0) return hipSuccess;
  const int max_block = cfg.variant >= 5 ? 512 : 256;
  if (cfg.block < 64 || cfg.block > max_block || cfg.block % 64 != 0 || cfg.tz < 1) return hipErrorInvalidValue;
  if (code < 0 || code > (BF16 | W12 | ONE)) return hipErrorInvalidValue;
  const int w = code & (W12 | ONE);
  switch (vprec(code)) {
    case F64: return launch_step_f64(w, width, cfg, groups, n_groups, tile_base, n_tiles, in, out, alpha, beta, lds, stream);
    case F32: return launch_step_f32(w, width, cfg, groups, n_groups, tile_base, n_tiles, in, out, alpha, beta, lds, stream);
    case F16S: return launch_step_f16s(w, width, cfg, groups, n_groups, tile_base, n_tiles, in, out, alpha, beta, lds, stream);
    default: return launch_step_bf16(w, width, cfg, groups, n_groups, tile_base, n_tiles, in, out, alpha, beta, lds, stream);
  }
}

hipError_t launch_build(int code, const void* U, const int32_t L[4], int t_first, int slot_first, int n_slices,
                        void* W, hipStream_t s) {
  const int64_t V3 = (int64_t)L[0] * L[1] * L[2];
  const int64_t Vp = padded_sites(V3);
  if (n_slices <= 0 || V3 <= 0) return hipSuccess;
  if (code < 0 || code > (BF16 | W12 | ONE)) return hipErrorInvalidValue;
  // workgroups per slice: a workgroup never spans two slices
  const int64_t per_slice = (V3 + kBuildSites * kBuildWaves - 1) / (kBuildSites * kBuildWaves);
  const int64_t blocks = per_slice * n_slices;
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks);
  const double2* u = static_cast<const double2*>(U);
  char* w = static_cast<char*>(W);
#define TL_BUILD(C) \
  case C: build_twolinks_kernel<C><<<grid, 64 * kBuildWaves, 0, s>>>(u, L[0], L[1], L[2], t_first, slot_first, (int)per_slice, w, Vp); break;
  switch (code) {
    TL_BUILD(F64)
    TL_BUILD(F32)
    TL_BUILD(F16S)
    TL_BUILD(BF16)
    TL_BUILD(F64 | W12)
    TL_BUILD(F32 | W12)
    TL_BUILD(F16S | W12)
    TL_BUILD(BF16 | W12)
    TL_BUILD(F64 | ONE)
    TL_BUILD(F32 | ONE)
    TL_BUILD(F16S | ONE)
    TL_BUILD(BF16 | ONE)
    TL_BUILD(F64 | W12 | ONE)
    TL_BUILD(F32 | W12 | ONE)
    TL_BUILD(F16S | W12 | ONE)
    TL_BUILD(BF16 | W12 | ONE)
    default: return hipErrorInvalidValue;
  }
#undef TL_BUILD
  return hipGetLastError();
}

hipError_t launch_pack(int prec, const void* nat, char* packed, const int64_t* rhs_off, int n_rhs, int64_t V3,
                       int64_t Vp, hipStream_t s) {
  if (n_rhs <= 0 || V3 <= 0) return hipSuccess;
  const dim3 grid((unsigned)((V3 + 255) / 256), (unsigned)n_rhs);
  const double2* n = static_cast<const double2*>(nat);
  switch (prec) {
    case F64: pack_kernel<F64><<<grid, 256, 0, s>>>(n, packed, rhs_off, V3, Vp); break;
    case F32: pack_kernel<F32><<<grid, 256, 0, s>>>(n, packed, rhs_off, V3, Vp); break;
    case F16S: pack_kernel<F16S><<<grid, 256, 0, s>>>(n, packed, rhs_off, V3, Vp); break;
    case BF16: pack_kernel<BF16><<<grid, 256, 0, s>>>(n, packed, rhs_off, V3, Vp); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_unpack(int prec, const char* packed, void* nat, const int64_t* rhs_off, int n_rhs, int64_t V3,
                         int64_t Vp, hipStream_t s) {
  if (n_rhs <= 0 || V3 <= 0) return hipSuccess;
  const dim3 grid((unsigned)((V3 + 255) / 256), (unsigned)n_rhs);
  double2* n = static_cast<double2*>(nat);
  switch (prec) {
    case F64: unpack_kernel<F64><<<grid, 256, 0, s>>>(packed, n, rhs_off, V3, Vp); break;
    case F32: unpack_kernel<F32><<<grid, 256, 0, s>>>(packed, n, rhs_off, V3, Vp); break;
    case F16S: unpack_kernel<F16S><<<grid, 256, 0, s>>>(packed, n, rhs_off, V3, Vp); break;
    case BF16: unpack_kernel<BF16><<<grid, 256, 0, s>>>(packed, n, rhs_off, V3, Vp); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int64_t red_partials_doubles(int n_rhs, int64_t max_v3) {
  const int64_t nb = std::max<int64_t>(1, (max_v3 + kRedSitesPerBlock - 1) / kRedSitesPerBlock);
  return 2 * nb * std::max(n_rhs, 1);
}

namespace {

template <class F>
hipError_t reduce_with(int kind, int prec, const char* a, const char* b, F f, int n_rhs, int64_t max_v3,
                       double* partials, double* out, hipStream_t s) {
  if (n_rhs <= 0 || max_v3 <= 0) return hipSuccess;
  if (kind == 2) {
    const dim3 grid((unsigned)((max_v3 + kRedBlock - 1) / kRedBlock), (unsigned)n_rhs);
    switch (prec) {
      case -1: site_norm_kernel<NatLoad><<<grid, kRedBlock, 0, s>>>(a, f, out); break;
      case F64: site_norm_kernel<PackedLoad<F64>><<<grid, kRedBlock, 0, s>>>(a, f, out); break;
      case F32: site_norm_kernel<PackedLoad<F32>><<<grid, kRedBlock, 0, s>>>(a, f, out); break;
      case F16S: site_norm_kernel<PackedLoad<F16S>><<<grid, kRedBlock, 0, s>>>(a, f, out); break;
      case BF16: site_norm_kernel<PackedLoad<BF16>><<<grid, kRedBlock, 0, s>>>(a, f, out); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  const int nb = (int)((max_v3 + kRedSitesPerBlock - 1) / kRedSitesPerBlock);
  const dim3 grid((unsigned)nb, (unsigned)n_rhs);
  switch (prec) {
    case -1: reduce_partial_kernel<NatLoad><<<grid, kRedBlock, 0, s>>>(kind, a, b, f, partials); break;
    case F64: reduce_partial_kernel<PackedLoad<F64>><<<grid, kRedBlock, 0, s>>>(kind, a, b, f, partials); break;
    case F32: reduce_partial_kernel<PackedLoad<F32>><<<grid, kRedBlock, 0, s>>>(kind, a, b, f, partials); break;
    case F16S: reduce_partial_kernel<PackedLoad<F16S>><<<grid, kRedBlock, 0, s>>>(kind, a, b, f, partials); break;
    case BF16: reduce_partial_kernel<PackedLoad<BF16>><<<grid, kRedBlock, 0, s>>>(kind, a, b, f, partials); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  reduce_finish_kernel<<<(n_rhs + 63) / 64, 64, 0, s>>>(kind, partials, nb, n_rhs, out);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_reduce(int kind, int prec, const char* a, const char* b, const RedField* f, int n_rhs,
                         int64_t max_v3, double* partials, double* out, hipStream_t s) {
  return reduce_with(kind, prec, a, b, TableFields{f}, n_rhs, max_v3, partials, out, s);
}

// ------------------------------------------------------------------ no-allocation reductions

// Partial sums of tl_reduce_noalloc: a fixed device array, one copy per device, held until
// the process ends.  Host code never passes the array's name to a kernel (that is a host-side
// stand-in, not a device address): it uses the address hipGetSymbolAddress gives on each
// device, looked up once per device when a context is created there.
static __device__ __align__(256) double scratch[kNoallocPartials];

namespace {
std::mutex g_noalloc_mu;
std::map<int, double*> g_noalloc_ptr;   // device -> address of its copy of `scratch`
}  // namespace

hipError_t noalloc_scratch_init(int device) {
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (g_noalloc_ptr.count(device)) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) return e != hipSuccess ? e : hipErrorInvalidSymbol;
  g_noalloc_ptr[device] = static_cast<double*>(p);
  return hipSuccess;
}

double* noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  auto it = g_noalloc_ptr.find(device);
  return it == g_noalloc_ptr.end() ? nullptr : it->second;
}

hipError_t launch_reduce_flat(int kind, const void* psi, const void* phi, int64_t n_sites, int n_rhs,
                              double* partials, double* out, hipStream_t s) {
  return reduce_with(kind, -1, static_cast<const char*>(psi), static_cast<const char*>(phi), FlatFields{n_sites},
                     n_rhs, n_sites, partials, out, s);
}

hipError_t launch_stream(void* buf, int64_t n_words, int n_in, int kinds, int grid, hipStream_t s) {
  if (n_words <= 0 || n_in < 1 || grid < 1) return hipErrorInvalidValue;
  const v4f* in = static_cast<const v4f*>(buf);
  v4f* out = static_cast<v4f*>(buf) + (int64_t)n_in * n_words;
  switch (kinds & 3) {
    case 0: stream_kernel<false, false><<<grid, 256, 0, s>>>(in, n_in, out, n_words); break;
    case 1: stream_kernel<true, false><<<grid, 256, 0, s>>>(in, n_in, out, n_words); break;
    case 2: stream_kernel<false, true><<<grid, 256, 0, s>>>(in, n_in, out, n_words); break;
    default: stream_kernel<true, true><<<grid, 256, 0, s>>>(in, n_in, out, n_words); break;
  }
  return hipGetLastError();
}

hipError_t launch_compare(const char* a, const char* b, int64_t n_bytes, int* flag, hipStream_t s) {
  const int64_t n16 = n_bytes / 16;
  const int64_t tail = n_bytes - n16 * 16;
  compare_kernel<<<1024, 256, 0, s>>>(reinterpret_cast<const uint4*>(a), reinterpret_cast<const uint4*>(b), n16,
                                      reinterpret_cast<const unsigned char*>(a) + n16 * 16,
                                      reinterpret_cast<const unsigned char*>(b) + n16 * 16, tail, flag);
  return hipGetLastError();
}

}  // namespace tl
