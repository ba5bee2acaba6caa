// Internal declarations shared by the kernels (tl_kernels.hip) and the host
// runtime (tl_runtime.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace tl {

// Storage precisions (same values as TL_F64 ... TL_BF16 in twolink.h).
enum Prec : int { F64 = 0, F32 = 1, F16S = 2, BF16 = 3 };

// Format codes: a precision, | W12 for the twelve-real link form (first two
// rows stored, third rebuilt), | ONE for a field of one-links U_mu(x) (the
// one-link Laplacian, hops of one site) instead of two-links W_mu(x) (hops
// of two sites).  Kernels are templated on the format code; colour vectors
// always use the format of vprec(code), link storage that of code & 7.
constexpr int W12 = 4;
constexpr int ONE = 8;
constexpr int vprec(int code) { return code & 3; }
constexpr bool is_w12(int code) { return (code & W12) != 0; }
constexpr bool is_one(int code) { return (code & ONE) != 0; }
constexpr int hop_of(int code) { return is_one(code) ? 1 : 2; }

// Packed link field: per slot, per direction mu, per site, kWBytes[code]
// bytes split into planes of vector words (see tl_format.h).  Packed colour
// vectors: per right-hand side, per site, kVBytes[code] bytes, also in planes.
constexpr int kWBytes[16] = {144, 72, 40, 36, 96, 48, 24, 24, 144, 72, 40, 36, 96, 48, 24, 24};
constexpr int kVBytes[16] = {48, 24, 16, 12, 48, 24, 16, 12, 48, 24, 16, 12, 48, 24, 16, 12};

// Plane length: sites per plane, rounded up so every plane starts 256-byte aligned.
inline int64_t padded_sites(int64_t v3) { return (v3 + 63) / 64 * 64; }

// A set of right-hand sides on one time slice of one lattice that share the
// two-link loads of a smearing step, plus the geometry of its tiles.
struct StepGroup {
  const char* W;          // packed two-link slot of the slice (direction x block)
  int64_t w_mu_stride;    // bytes between direction blocks (Vp * kWBytes)
  int64_t psi_off;        // byte offset of the group's first RHS in the resident buffers
  int64_t rhs_stride;     // bytes between consecutive RHS of the group (Vp * kVBytes)
  int32_t Lx, Ly, Lz;
  int32_t Vp;             // plane length (padded sites)
  int32_t nr;             // RHS in the group
  int32_t n_xy_tiles;     // ceil(Lx*Ly / block)
  int32_t n_z_tiles;      // ceil(Lz / tz)
  int32_t tile_begin;     // work-list index of the group's first tile
  int32_t rows;           // variants 5-7: full rows of the xy plane per tile (divides Ly)
};

// Launch configuration of the step kernel.
struct StepConfig {
  int variant;   // 0: one site per thread per z plane, neighbours through the caches
                 // 1: z-marching with a register ring of colour vectors for the z hops
                 // 2: z-marching with rings of colour vectors and z two-links, chunks
                 //    marching in alternating directions
                 // 3: as 2, with each plane's in-plane hops computed when the plane is
                 //    first loaded (every plane read from memory once)
                 // 4: as 0 with the direction loop rolled (fewer registers, more waves)
                 // 5: as 2, with tiles of full rows whose in-plane neighbours are
                 //    exchanged through LDS (fewer vector-memory instructions)
                 // 6: as 5, marching chains of planes z, z+2, ... (smaller rings; the
                 //    in-plane two-links are loaded before the LDS barrier)
                 // 7: as 6, software-pipelined: each plane step issues the next step's
                 //    loads into the registers its own arithmetic has just freed
                 // 8: two steps per launch: tiles of k rows of one y chain (rows y, y+2, ...),
                 //    the first step also on one chain row beyond each side, its result
                 //    kept in LDS for the second (an odd step count ends with one launch
                 //    of a one-step tiling)
  int block;     // threads per workgroup (xy sites per tile; variants 5-7: an upper bound)
  int tz;        // z planes per tile
  int grid;      // workgroups; <= 0 means one workgroup per tile
  int nt;        // 1: nontemporal output stores (pays when a step's working set exceeds the
                 // Infinity Cache; costs when the next step could have re-read it from there)
  int flip;      // 1: odd steps of a sequence run reversed (tile order and march directions),
                 // so a step starts on the planes the previous step touched last, which are
                 // still in the Infinity Cache when a step's working set exceeds it
  int rev;       // set per launch: this launch runs reversed
  int rows64;    // variant 8, set with the work list: every group's rows are 64 sites long
  int width;     // RHS per step group in the work list (0: the plan's groups, up to four RHS of a
                 // slice sharing each two-link load; 1: every RHS its own tiles, more parallel
                 // work for small lattices, the two-links loaded once per RHS)
};

// Rows per tile of variants 5-7 for an Lx x Ly plane and a block size: the largest divisor of Ly
// with rows * Lx <= block and rows >= 4 (0 if there is none).
inline int lds_rows(int Lx, int Ly, int block) {
  for (int r = block / Lx; r >= 4; r--)
    if (Ly % r == 0) return r;
  return 0;
}

// Dynamic LDS bytes variants 5-7 need for a group: two buffers of (rows + 4) rows of R vectors.
inline int64_t lds_bytes(int code, int R, int Lx, int rows) {
  return 2LL * (rows + 4) * Lx * R * 6 * (vprec(code) == F64 ? 8 : 4);
}

// Dynamic LDS bytes variant 8 needs for a group: two input planes of k + 4 rows and two
// step-one planes of k + 2 rows of R vectors (FP32 planes padded to an even entry count).
inline int64_t lds_bytes_fuse2(int code, int R, int Lx, int k) {
  auto plane = [&](int64_t rn) { return vprec(code) == F64 ? 48 * rn : 24 * ((rn + 1) & ~int64_t(1)); };
  return 2 * (plane((int64_t)R * (k + 4) * Lx) + plane((int64_t)R * (k + 2) * Lx));
}

// Chain rows per tile of variant 8 for an Lx x Ly plane of format `code` with R RHS per group
// and a block size: the largest k that divides the y chain's length (Ly / 2 for two-link hops
// and even Ly, else Ly) with (k + 2) * Lx <= block and LDS within lds_max (0 if there is none).
inline int fuse_rows(int code, int R, int Lx, int Ly, int block, int64_t lds_max) {
  const int ylen = (hop_of(code) == 2 && !(Ly & 1)) ? Ly / 2 : Ly;
  for (int k = (block / Lx - 2 < ylen ? block / Lx - 2 : ylen); k >= 1; k--)
    if (ylen % k == 0 && lds_bytes_fuse2(code, R, Lx, k) <= lds_max) return k;
  return 0;
}

// Raise the dynamic-LDS limit of the LDS-staged step kernels (once per device, before any capture).
hipError_t init_kernel_attributes();

// psi_out = alpha psi_in + beta sum_hops on every tile in [tile_base, tile_base + n_tiles).
// code: format code (precision, optionally | W12).  lds: dynamic LDS bytes for variants
// 5-7 (max over the groups), 0 otherwise.
hipError_t launch_step(int code, int width, const StepConfig& cfg, const StepGroup* groups,
                       int n_groups, int tile_base, int n_tiles, const char* in, char* out,
                       double alpha, double beta, int64_t lds, hipStream_t stream);

// The step kernels of one precision (one translation unit each); form = code & (W12 | ONE).
#define TL_STEP_DECL(name)                                                                              \
  hipError_t launch_step_##name(int form, int width, const StepConfig& cfg, const StepGroup* groups,     \
                                int n_groups, int tile_base, int n_tiles, const char* in, char* out,    \
                                double alpha, double beta, int64_t lds, hipStream_t stream);           \
  hipError_t step_attributes_##name();
TL_STEP_DECL(f64)
TL_STEP_DECL(f32)
TL_STEP_DECL(f16s)
TL_STEP_DECL(bf16)
#undef TL_STEP_DECL

// W slots slot_first .. slot_first+n-1 from slices t_first .. t_first+n-1, in format `code`:
// two-links W_mu(x) = U_mu(x) U_mu(x+mu^), or the links U_mu(x) themselves when is_one(code).
hipError_t launch_build(int code, const void* U, const int32_t L[4], int t_first, int slot_first, int n,
                        void* W, hipStream_t stream);

// Natural complex128 [rhs][V3][3] <-> packed resident field.  rhs_off[r] is
// the byte offset of RHS r in the packed buffer (device array).
hipError_t launch_pack(int prec, const void* nat, char* packed, const int64_t* rhs_off_dev,
                       int n_rhs, int64_t V3, int64_t Vp, hipStream_t stream);
hipError_t launch_unpack(int prec, const char* packed, void* nat, const int64_t* rhs_off_dev,
                         int n_rhs, int64_t V3, int64_t Vp, hipStream_t stream);

// Description of one RHS for the reductions.
struct RedField {
  int64_t off;      // byte offset (packed) or element offset (natural) of the RHS
  int64_t off2;     // same for the second field of a dot product
  int64_t V3;       // sites
  int64_t Vp;       // plane length (packed)
  int64_t out_off;  // first output index of this RHS (site norms)
};

// kind: 0 norm2, 1 dot, 2 site norms.  prec = -1 selects natural complex128
// fields.  partials: device scratch of at least red_partials_doubles(n_rhs) doubles.
int64_t red_partials_doubles(int n_rhs, int64_t max_v3);
hipError_t launch_reduce(int kind, int prec, const char* a, const char* b, const RedField* fields_dev,
                         int n_rhs, int64_t max_v3, double* partials, double* out, hipStream_t stream);

// No-allocation reductions (tl_reduce_noalloc): natural complex128 fields [n_rhs][n_sites][3]
// reduced with their first-pass partial sums in a fixed per-device array of kNoallocPartials
// doubles.  noalloc_scratch_init looks up this device's copy (the device must be current);
// noalloc_scratch returns it, or NULL before the lookup.
constexpr int64_t kNoallocPartials = 2 * 65536;
hipError_t noalloc_scratch_init(int device);
double* noalloc_scratch(int device);
hipError_t launch_reduce_flat(int kind, const void* psi, const void* phi, int64_t n_sites, int n_rhs,
                              double* partials, double* out, hipStream_t stream);

// Streaming probe over buf cut into n_in + 1 planes of n_words 16-byte words: plane n_in =
// sum of planes 0 .. n_in - 1.  kinds bit 0: nontemporal loads, bit 1: nontemporal stores.
hipError_t launch_stream(void* buf, int64_t n_words, int n_in, int kinds, int grid, hipStream_t stream);

// flag[0] = 1 if the n_bytes at a and b differ anywhere (flag must be cleared by the caller).
hipError_t launch_compare(const char* a, const char* b, int64_t n_bytes, int* flag, hipStream_t stream);

}  // namespace tl
