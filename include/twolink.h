/*
 * twolink.h -- C ABI of libtwolink.so: two-link staggered Gaussian smearing
 * on AMD Instinct MI355X (gfx950).
 *
 * Method (Gottlieb, Jeong, Strelchenko, arXiv:2301.05518, Sec. 2 and 3):
 *   two-link product    W_mu(x) = U_mu(x) U_mu(x+mu^),  mu = x, y, z
 *   two-link Laplacian  4 Lap psi(x) = sum_mu [W_mu(x) psi(x+2mu^)
 *                                       + W_mu^dag(x-2mu^) psi(x-2mu^)] - 6 psi(x)   (eq. tlLapl1)
 *   smearing            psi <- (1 + (sigma/n) Lap)^n psi                            (eq. tlSmear)
 * The Laplacian is three-dimensional: it acts on one time slice and never
 * hops in t.  Boundaries are periodic in x, y and z.  W is built once per
 * gauge field and reused for every source and sink (Sec. 3).
 *
 * Conventions common to every entry point
 * ---------------------------------------
 * - Return value: TL_OK (0) or a negative TL_ERR_* code.  tl_last_error()
 *   gives a message.  Argument errors are detected before any device work
 *   is queued, and nothing is written in that case.  No C++ exception
 *   crosses this interface.
 * - Asynchrony: device work is queued on the context's stream and the call
 *   returns without waiting, unless stated otherwise.  Errors raised by the
 *   device afterwards surface at tl_sync() or at a later call.
 * - Ownership: the caller owns every buffer passed in (gauge field, two-link
 *   field, colour-vector fields, outputs).  The library never frees them and
 *   keeps no pointer to them after the call returns, except that a plan
 *   (tl_plan_*) keeps the job pointers given to tl_plan_create until
 *   tl_plan_destroy.  Library-internal memory (resident packed fields,
 *   work lists, reduction partials, scratch) belongs to the context or plan.
 * - "device" pointers are HIP device memory of the context's device;
 *   "host" pointers are ordinary host memory read during the call.
 * - Geometry: tl_geom.L = {Lx, Ly, Lz, Lt}, every extent in [1, 4096] and
 *   Lx*Ly*Lz <= 2^27.
 * - Natural layouts (complex128 = two doubles, real part first):
 *     gauge field U       [Lt][Lz][Ly][Lx][mu=0..3][a][b]   mu = x, y, z, t
 *                         U_mu(x) transports a vector from x+mu^ to x.
 *     colour vectors psi  [n_rhs][Lz][Ly][Lx][c]            one slice per RHS
 *   The two-link field W is an opaque packed buffer in the storage
 *   precision it was built in; size it with tl_twolinks_bytes().
 * - Storage precisions: TL_F64 (FP64 storage and arithmetic), TL_F32,
 *   TL_F16S (IEEE half times one FP32 scale per site), TL_BF16; the last
 *   three use FP32 arithmetic.  The two-link product is always formed in
 *   FP64 and rounded to the storage precision when stored.  Reductions
 *   accumulate in FP64.
 * - Twelve-real two-links: every `prec` argument may carry TL_W12
 *   (e.g. TL_F32 | TL_W12).  The two-link field then stores only the first
 *   two rows of each W_mu(x) and the kernels rebuild the third as the complex
 *   conjugate of the cross product of the first two, which is exact for
 *   special unitary matrices: a two-link of SU(3) links is in SU(3), but
 *   one of links that are not special unitary (e.g. gauge-smeared links
 *   without reunitarisation, end of Sec. 2) is not, and for those the
 *   results are wrong -- the caller guarantees SU(3) links.
 *   Bytes per site and direction: 96 (F64), 48 (F32), 24 (F16S, BF16; the
 *   16-bit forms hold plain values with no scale, every entry of an SU(3)
 *   matrix having modulus <= 1).  Colour vectors keep the format of the
 *   precision.  A field built with TL_W12 must be used with TL_W12 and the
 *   same precision.
 * - One-link Gaussian smearing (Sec. 2, eq. gsmear and the rewriting that
 *   follows it): a `prec` carrying TL_ONELINK names a field of the links
 *   U_mu(x) themselves, packed by tl_pack_links in the same layout (and size)
 *   as a two-link field, and makes tl_laplacian apply the one-link Laplacian
 *   nabla^2 = H - 6 (hops of one site, no 1/4) and tl_smear / tl_plan_create
 *   apply (1 + (sigma/n) nabla^2)^n with 0 <= sigma/n <= 1/6.  The hopping
 *   form C (1 + alpha H)^n of eq. gsmear equals C (1 + 6 alpha)^n times this
 *   with sigma = n alpha / (1 + 6 alpha).  Only the step variants 0, 4 and 7
 *   run one-link fields (the autotuner restricts itself to them).
 */
#ifndef TWOLINK_H
#define TWOLINK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ codes */
enum {
    TL_OK = 0,
    TL_ERR_ARG = -1,         /* null pointer, bad count, bad flag or kind, aliasing */
    TL_ERR_SHAPE = -2,       /* geometry out of range, slice not present in W */
    TL_ERR_PRECISION = -3,   /* unknown storage precision */
    TL_ERR_DEVICE = -4,      /* no such device, or device work on a host-only context */
    TL_ERR_HIP = -5,         /* a HIP runtime call failed (message from the runtime) */
    TL_ERR_NOMEM = -6,       /* a library-internal allocation (device or host) failed */
    TL_ERR_UNSUPPORTED = -7  /* valid request this build does not implement */
};

enum { TL_F64 = 0, TL_F32 = 1, TL_F16S = 2, TL_BF16 = 3 };
enum { TL_W12 = 16 };   /* OR into a precision: twelve-real (two-row) link storage */
enum { TL_ONELINK = 32 };  /* OR into a precision: a one-link field and the one-link operators */

/* tl_smear / tl_plan_create flags */
enum {
    TL_PLAIN = 1u,      /* one right-hand side per launch, RHS in succession, eager launches */
    TL_GRAPH = 2u,      /* capture the n step launches in one HIP graph, replayed per run */
    TL_AUTOTUNE = 4u,   /* time the candidate tilings once and keep the fastest (cached per context;
                           with TL_PLAIN timed on one RHS of each lattice shape, weighted by the
                           shape's RHS count); for batched plans of two or more steps the
                           candidates include launches
                           that run two steps each (the first step's result kept on chip, rounded
                           to the storage precision exactly as a store would round it, so the
                           result is bit-identical to one step per launch) */
    TL_ONE_STEP = 8u    /* tune over tilings of one step per launch only (no two-step launches) */
};

/* reduction kinds.  TL_NORM2 and TL_DOT are the spatial sums over the sites x of one
 * time slice that make up a two-point correlation function C(t) (Sec. 1: C(t) sums the
 * product of the operator at (t, x) and its conjugate at the source over x; contracted
 * from smeared source and sink vectors it is such a slice sum of colour inner products);
 * TL_SITE_NORM is the per-site magnitude of a smeared source that Fig. 1 plots. */
enum {
    TL_NORM2 = 0,       /* per RHS: sum_x |psi(x)|^2                -> out[n_rhs] */
    TL_DOT = 1,         /* per RHS: sum_x phi(x)^dag psi(x)         -> out[2*n_rhs] (re, im) */
    TL_SITE_NORM = 2    /* per RHS and site: |psi(x)| (Fig. 1 quantity) -> out[n_rhs*V3] */
};

typedef struct { int32_t L[4]; } tl_geom;   /* Lx, Ly, Lz, Lt */

/* Counters of one context (filled by tl_get_stats). */
typedef struct {
    int64_t graphs_captured;   /* HIP graphs captured by the context's plans */
    int64_t tune_sweeps;       /* autotuning sweeps run (TL_AUTOTUNE with no cached result) */
    int64_t tune_hits;         /* plans whose tiling came from the tuning cache (memory or TL_TUNE_CACHE) */
    int64_t smear_plan_hits;   /* tl_smear(TL_GRAPH) calls served by a plan kept from an earlier call */
} tl_ctx_stats;

typedef struct tl_ctx tl_ctx;
typedef struct tl_plan tl_plan;

/* One lattice's share of a smearing batch. */
typedef struct {
    tl_geom g;
    const void *W;             /* device: two-link field built in the batch's precision */
    const int32_t *w_slices;   /* host: slice list W was built for; NULL = all Lt slices in order */
    int32_t n_w_slices;        /* entries in w_slices (ignored when w_slices is NULL) */
    int32_t n_rhs;             /* right-hand sides of this lattice, >= 1 */
    const int32_t *t_of_rhs;   /* host: time slice of each RHS, n_rhs entries, each in W */
    void *psi;                 /* device: complex128 [n_rhs][Lz][Ly][Lx][3], smeared in place */
} tl_job;

/* What a plan resolved to (filled by tl_plan_get_info). */
typedef struct {
    int32_t n_groups;          /* RHS groups: RHS of one slice that share each W load */
    int32_t group_width;       /* largest group */
    int32_t n_tiles;           /* work-list entries per step */
    int32_t variant;           /* step kernel variant (0 direct, 1-3 z-marching, 4 rolled, 5-7 LDS row
                                  tiles, 8 two steps per launch) */
    int32_t block;             /* threads per workgroup */
    int32_t tz;                /* z planes per tile */
    int32_t grid;              /* workgroups per step launch */
    int32_t nt;                /* 1: nontemporal output stores */
    int32_t flip;              /* 1: odd steps run in reversed tile and march order */
    int32_t launches_per_step; /* 1 for batched plans, n_groups for TL_PLAIN (launches of one
                                  step each; see steps_per_launch) */
    int32_t steps_per_launch;  /* 2 when each launch runs two steps (variant 8; an odd step count
                                  ends with one launch of a one-step tiling), else 1 */
    int32_t tile_width;        /* RHS per step group in the launches: group_width, or 1 when the
                                  tuned tiling gives every RHS its own tiles */
    int64_t rhs_sites;         /* sum over RHS of Lx*Ly*Lz */
    double bytes_per_step;     /* algorithmic bytes of one step: W once per group + psi in and out */
    double flops_per_step;     /* 444 per RHS-site-update */
    int64_t resident_bytes;    /* device memory the plan holds */
} tl_plan_info;

/* ---------------------------------------------------------------- context */

/* Library version, major*10000 + minor*100 + patch. */
int tl_version(void);

/*
 * Environment (read by the library):
 *   TL_TILE="variant,block,tz,grid[,nt[,flip[,width]]]"  fix the step tiling of every plan (no
 *                                    tuning); for profiling and sweeps.  width: RHS per step
 *                                    group (0 or absent: the plan's groups; 1: every RHS on its
 *                                    own tiles).  Variant 8 (two steps per launch) may name the
 *                                    one-step tiling an odd step count ends with after a ';'
 *                                    (default "0,256,4,0,0,0")
 *   TL_LOG=1                         print autotuning candidates to stderr
 *   TL_FAULT=alloc|launch            make internal allocations or launches fail
 *                                    (read at tl_create; exercises error paths)
 *   TL_TUNE_CACHE=<path>             a JSON file of autotuning results: read at tl_create,
 *                                    rewritten after every sweep, so that a later process
 *                                    skips the sweep for batch shapes already tuned (keys name
 *                                    the GPU architecture, precision, group width, launch mode
 *                                    and every group's extents and RHS count); an entry whose
 *                                    tiling the plan cannot run is dropped and tuned again
 */

/*
 * Create a context on HIP device `device`, queueing on `stream` (a
 * hipStream_t; NULL = the null stream).  device = -1 creates a host-only
 * context that validates arguments and answers size queries but returns
 * TL_ERR_DEVICE for any device work.  *out receives the context.
 */
int tl_create(tl_ctx **out, int device, void *stream);
int tl_destroy(tl_ctx *ctx);
/*
 * Queue the context's later work on `stream` (a hipStream_t of the context's
 * device; NULL = the null stream).  The new stream is made to wait (through an
 * event, without blocking the host) for everything already queued on the old
 * one, so library memory that earlier calls still use (context scratch, plan
 * buffers) is not overwritten by later calls; the caller's own work on either
 * stream is not otherwise ordered.  Plans created before the switch queue on the
 * new stream from then on.  TL_ERR_HIP if the runtime refuses the event.
 */
int tl_set_stream(tl_ctx *ctx, void *stream);
/* Block until the context's stream is idle; reports asynchronous device errors. */
int tl_sync(tl_ctx *ctx);
/* Message of the last failing call on ctx (ctx = NULL: last failure of tl_create on this thread). */
const char *tl_last_error(const tl_ctx *ctx);
/* The context's counters (TL_ERR_ARG for NULL arguments). */
int tl_get_stats(const tl_ctx *ctx, tl_ctx_stats *out);

/* ------------------------------------------------------------------ sizes */

/* TL_OK if g is a supported geometry, TL_ERR_SHAPE (or TL_ERR_ARG for NULL) otherwise. */
int tl_check_geom(const tl_geom *g);
/* Bytes of a two-link field for n_slices slices in precision prec (optionally | TL_W12; 0 on bad arguments). */
size_t tl_twolinks_bytes(const tl_geom *g, int prec, int n_slices);

/* ---------------------------------------------------------------- the path */

/*
 * Two-link product (Sec. 2; precomputed once per gauge field, Sec. 3):
 * W_mu(x) = U_mu(x) U_mu(x+mu^) for mu = x, y, z at every site of the listed
 * slices, formed in FP64 and stored in precision `prec` (| TL_W12: first two
 * rows only).
 *   U        device, complex128 natural gauge field of geometry g (only the
 *            spatial links of the listed slices are read)
 *   slices   host, n_slices slice indices, each in [0, Lt), no repeats;
 *            NULL = all Lt slices in order (n_slices must then be Lt or 0)
 *   W        device, tl_twolinks_bytes(g, prec, n_slices) bytes, written;
 *            slot j holds slice slices[j]
 */
int tl_build_twolinks(tl_ctx *ctx, const tl_geom *g, const void *U,
                      const int32_t *slices, int n_slices, int prec, void *W);

/*
 * One-link field for one-link Gaussian smearing (Sec. 2): the spatial links
 * U_mu(x), mu = x, y, z, of the listed slices, rounded to precision `prec`,
 * which must carry TL_ONELINK (and may carry TL_W12).  Arguments, layout and
 * size as for tl_build_twolinks; TL_ERR_PRECISION without TL_ONELINK (and
 * tl_build_twolinks refuses TL_ONELINK).
 */
int tl_pack_links(tl_ctx *ctx, const tl_geom *g, const void *U,
                  const int32_t *slices, int n_slices, int prec, void *W);

/*
 * One application of the two-link Laplacian of eq. tlLapl1 (including the
 * factor 1/4 and the -6 term) on time slice t:  out = Lap in.
 *   W, w_slices, n_w_slices  as in tl_job; t must be one of W's slices
 *   in, out  device complex128 [Lz][Ly][Lx][3]; out must not overlap in
 * `in` is rounded to the storage precision first; the arithmetic is FP64 for
 * TL_F64 and FP32 otherwise; the result is rounded to the storage precision
 * and then widened to complex128.  Uses context scratch memory.  With
 * TL_ONELINK in prec (W from tl_pack_links): the one-link Laplacian
 * nabla^2 = H - 6 of Sec. 2 instead.
 */
int tl_laplacian(tl_ctx *ctx, const tl_geom *g, const void *W, const int32_t *w_slices,
                 int n_w_slices, int prec, int t, const void *in, void *out);

/*
 * Smearing of eq. tlSmear, psi <- (1 + (sigma/n) Lap)^n psi with n = n_steps,
 * applied in place to every right-hand side of every job on its own slice.
 * Jobs may have different geometries (uneven batch).  Equivalent to
 * tl_plan_create + load + run + store + destroy, except with TL_GRAPH: the
 * context then keeps the plan (resident buffers, work list, tiling, captured
 * graph) of its 4 most recent distinct calls, keyed by everything the call
 * passes (device pointers, geometries, slice lists, n, sigma, precision,
 * flags), and a repeated call replays the kept graph without capturing; the
 * kept plans hold device memory until they are displaced or tl_destroy.
 * Requires n_steps >= 0, finite sigma with 0 <= sigma/n_steps <= 2/3 (the step
 * is then a contraction).
 */
int tl_smear(tl_ctx *ctx, const tl_job *jobs, int n_jobs, int n_steps, double sigma,
             int prec, unsigned flags);

/* ------------------------------------------------------- resident plans */

/*
 * A plan holds the batch's colour vectors resident on the device in packed
 * storage precision, the step work list, the tuned tiling and (TL_GRAPH) the
 * captured step graph, so that repeated runs pay none of that again.
 * The jobs array (and the host arrays it points to) is copied; the device
 * pointers in it (W, psi) must stay valid until tl_plan_destroy.
 */
int tl_plan_create(tl_ctx *ctx, const tl_job *jobs, int n_jobs, int n_steps, double sigma,
                   int prec, unsigned flags, tl_plan **out);
/* Pack every job's psi (complex128) into the resident buffer (rounds to the storage precision). */
int tl_plan_load(tl_plan *plan);
/* n_steps smearing steps on the resident buffer (eq. tlSmear applied n_steps times; with a
   two-step tiling, n_steps / 2 launches plus one one-step launch when n_steps is odd). */
int tl_plan_run(tl_plan *plan);
/* Unpack the resident buffer into every job's psi (complex128). */
int tl_plan_store(tl_plan *plan);
/*
 * FP64 reduction of the resident fields (decoded from storage precision),
 * deterministic summation order: the slice sums of a two-point correlation
 * function C(t) (Sec. 1) and the per-site magnitude of Fig. 1.  kind: TL_NORM2, TL_DOT (needs `other`, a
 * plan with the same jobs' shapes; <other, this> per RHS), TL_SITE_NORM.
 * out: device doubles, sized as for the kind (RHS in the order of the jobs).
 */
int tl_plan_reduce(tl_plan *plan, int kind, const tl_plan *other, double *out);
/* Average device time of one step kernel launch over `reps` back-to-back
 * runs of n_steps steps each (after one untimed run that tunes and captures),
 * measured with HIP events on the context's stream (blocks the host).  The
 * resident fields are smeared reps + 1 more times: tl_plan_load before using
 * results again. */
int tl_plan_time(tl_plan *plan, int reps, double *ms_per_step);
int tl_plan_get_info(const tl_plan *plan, tl_plan_info *info);

/*
 * Streaming bandwidth probe (a measurement utility beside the method): the HBM
 * rate a plain stream reaches with the read/write mix of a smearing step, as a
 * ceiling to set the step kernel's rate against (memory bandwidth bounds the
 * smearing iterations, Sec. 5).  buf (device, `bytes` long, 256-byte aligned)
 * is cut into n_in + 1 equal planes of 16-byte words; one launch writes the last
 * plane as the FP32 sum of the first n_in (n_in bytes read per byte written).
 * kinds: bit 0 nontemporal loads, bit 1 nontemporal stores (the step kernels
 * load cached and store nontemporally); grid: workgroups of 256 threads (0 =
 * 16 per compute unit).  Runs reps + 1 launches, the first untimed, and writes
 * the average duration of one launch in ms to *ms (HIP events on the context's
 * stream; blocks the host).  buf's contents are overwritten.
 */
int tl_stream_time(tl_ctx *ctx, void *buf, int64_t bytes, int n_in, int kinds, int grid, int reps,
                   double *ms);
int tl_plan_destroy(tl_plan *plan);

/* -------------------------------------------------------- reductions */

/*
 * FP64 reductions of natural complex128 fields psi, phi [n_rhs][n_sites][3]
 * (device): per RHS the slice sum of a two-point correlation function C(t)
 * (Sec. 1; TL_NORM2, TL_DOT) or the per-site magnitude plotted in Fig. 1
 * (TL_SITE_NORM).  kind as above; phi only for TL_DOT (<phi, psi> per RHS).
 * The fields are flat: any set of sites (one slice, several, a sub-volume),
 * since a sum over sites needs no geometry.
 * out: device doubles (n_rhs, 2*n_rhs or n_rhs*n_sites entries), written.
 * Errors: TL_ERR_ARG for an unknown kind, NULL field or output, n_sites < 1 or
 * n_rhs < 1; TL_ERR_SHAPE for n_sites > 2^40.  Uses context scratch memory
 * (the partial sums), grown with hipMalloc when too small.
 */
int tl_reduce(tl_ctx *ctx, int kind, int64_t n_sites, int n_rhs, const void *psi,
              const void *phi, double *out);

/*
 * tl_reduce without any allocation, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Arguments, results (bit for bit) and errors as for
 * tl_reduce, plus: TL_ERR_SHAPE, before any device work, when the first pass
 * needs more partial sums than the fixed area holds, i.e. for TL_NORM2 and
 * TL_DOT n_rhs * ceil(n_sites / 4096) must not exceed 65536 (TL_SITE_NORM has
 * no limit); TL_ERR_HIP if the area's address could not be looked up when the
 * context was created.  The partial sums live in one fixed device array of
 * 1 MiB per device (held until the process ends), shared by every context and
 * call on that device: calls that overlap on one device (other streams, other
 * threads) race and give wrong results; calls queued on one stream are
 * ordered.  No host-to-device copy, no hipMalloc, no hipFree, no memset.
 */
int tl_reduce_noalloc(tl_ctx *ctx, int kind, int64_t n_sites, int n_rhs, const void *psi,
                      const void *phi, double *out);

#ifdef __cplusplus
}
#endif

#endif /* TWOLINK_H */
