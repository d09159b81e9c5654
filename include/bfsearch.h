/*
 * bfsearch.h -- C ABI of the MI355X matched-filter hot path of butterfly
 * filtering (van Putten, "Deep searches for broadband extended
 * gravitational-wave emission bursts by heterogeneous computing",
 * arXiv:1708.01609).
 *
 * Problem statement (Sec. 3): a real strain segment y of N samples is
 * correlated against a bank of real chirp templates w_j (Eq. 3), evaluated by
 * the three-step FFT correlation of Eq. (5): forward real FFTs, the product
 * conj(W) * Y, an inverse FFT.  Each correlation's standard deviation sigma
 * (Eq. 6) is predicted from the spectrum by Parseval's theorem (Eq. 7) before
 * the inverse transform, and only the tails |rho_n| > kappa * sigma (Eq. 9,
 * on the absolute value) are compacted on the device and returned to the host
 * (Sec. 3.2-3.3, "gather all hits" mode).
 *
 * Conventions fixed by this library:
 *   rho_sj[n] = sum_{m<L} w_j[m] * y_s[(n + m) mod N],  n = 0..N-1
 *     (circular: the template is zero-padded to N, Sec. 3.2 step (ii)),
 *   sigma_sj  = sqrt(sum_n rho_sj[n]^2 / N)      (Eq. 6, RMS about zero),
 *   computed as (1/N) sqrt(|C_0|^2 + |C_{N/2}|^2 + 2 sum_{k=1}^{N/2-1} |C_k|^2)
 *     with C = conj(W) Y (the exact form of Eq. 7 for any real input),
 *   tail = (s, j, n, rho) for every |rho_sj[n]| > kappa * sigma_sj (strict).
 *   Grid templates: w_j[m] = h[m] cos(2 pi (f0 t + fdot t^2 / 2)), t = m/fs,
 *   h the symmetric Hann window, normalised to sum w^2 = 1; template id
 *   j = i_f0 * n_fdot + i_fdot over inclusive linspace grids; duration
 *   tau[j % n_tau], L = nearest integer to tau * fs (ties to even).
 *
 * Errors: every call returns a bfs_status; nothing throws across the ABI.
 * Argument checks happen before any HIP call, so an invalid call returns
 * BFS_ERR_INVALID_ARG without touching the device.
 *
 * Threading: a plan is immutable after bfsearch_plan and may be used by
 * several threads issuing bfsearch_filter on different streams.  A job is
 * used by one thread at a time.
 */
#ifndef BFSEARCH_H
#define BFSEARCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BFS_OK = 0,
  BFS_ERR_INVALID_ARG = -1,   /* bad descriptor, size, pointer or length */
  BFS_ERR_OUT_OF_MEMORY = -2, /* HBM budget or device allocation exceeded; nothing kept */
  BFS_ERR_HIP = -3,           /* a HIP runtime call failed */
  BFS_ERR_TAIL_OVERFLOW = -4, /* more tails than capacity; totals stay exact */
  BFS_ERR_UNSUPPORTED = -5,   /* valid request outside the built kernel set */
  BFS_ERR_SCRATCH_LIMIT = -6  /* bfsearch_filter_noalloc: the segments' spectra do
                                 not fit the fixed scratch area */
} bfs_status;

typedef enum {
  BFS_FP64 = 0,      /* samples, spectra and FFTs in FP64 */
  BFS_FP32 = 1,      /* FP32 samples, spectra and FFTs; sigma and norms in FP64 */
  BFS_FP32_W16F = 2, /* as BFS_FP32, template spectra stored as FP16 */
  BFS_FP32_W16B = 3  /* as BFS_FP32, template spectra stored as BF16 */
} bfs_precision;

/* Plan flags. */
#define BFS_PLAN_GRAPH 1u    /* capture each job shape once as a HIP graph and
                                replay it (fewer launches per filter call) */
#define BFS_PLAN_AUTOTUNE 2u /* at plan time, time every kernel candidate and
                                every segment tile of each length on the
                                resident bank and keep the fastest (default:
                                the first candidate; the tile whose segment
                                spectra fill half an XCD's L2) */

#define BFS_PLAN_PROJECT 4u  /* per-lag max projection (Sec. 3.3, Eqs. 13-17)
                                instead of the tail list: see
                                bfsearch_fetch_projection */
#define BFS_PLAN_SYMMETRIC 8u /* grid templates symmetric in time: the chirp
                                 plus its time reversal, x[m] + x[L-1-m],
                                 normalised after the sum (the paper's bank
                                 shape, Fig. 2 caption), for ascending and
                                 descending chirps alike */

#define BFS_PLAN_PAIRS 16u    /* detector pairs (Sec. 3.2 step (i), Sec. 5): the
                                 segments of a filter call come as time-aligned
                                 channel pairs, pair p's channels at segments 2p
                                 and 2p + 1 (equal lengths).  Each (pair, template)
                                 is correlated through one complex inverse
                                 transform carrying both channels (real part:
                                 channel 2p, imaginary part: channel 2p + 1);
                                 tails, sigma and projections are reported per
                                 segment as for single segments.  Lengths whose
                                 transform the library splits (2^17 FP32, 2^14
                                 FP64) are BFS_ERR_UNSUPPORTED */

#define BFS_PLAN_FUSED 32u    /* fused synthesis: keep no template bank; each
                                 correlation synthesises its chirp on chip (FP64
                                 phase and taper), transforms it and goes on as
                                 with a resident bank (Sec. 3.2 steps (ii)-(iv)
                                 with step (ii) made per correlation).  Grid
                                 plans of BFS_FP32 precision without
                                 BFS_PLAN_PAIRS, at lengths 2^10, 2^13 and 2^16
                                 (else BFS_ERR_UNSUPPORTED).  Such a plan whose
                                 resident bank would exceed the HBM budget takes
                                 this form without the flag.  bfsearch_plan_spectra
                                 is BFS_ERR_UNSUPPORTED for it */

typedef struct bfs_plan bfs_plan; /* opaque: resident template banks, tables */
typedef struct bfs_job bfs_job;   /* opaque: one bfsearch_filter call */

/* One tail record (16 bytes).  rho is the correlation value rho_sj[lag] of
 * the convention above (not divided by sigma), FP32: the FP32 path's own
 * precision; FP64 plans round theirs (bfs_tail64 keeps it). */
typedef struct {
  uint32_t segment;
  uint32_t template_id;
  uint32_t lag;
  float rho;
} bfs_tail;

/* The same with an FP64 rho (24 bytes): the record the FP64 path writes. */
typedef struct {
  uint32_t segment;
  uint32_t template_id;
  uint32_t lag;
  uint32_t reserved;
  double rho;
} bfs_tail64;

/* One entry of the per-lag max projection (16 bytes): at lag `lag` of
 * segment `segment`, the template with the largest |rho| / sigma among those
 * whose |rho| exceeds kappa * sigma; snr = rho / sigma of that template, sign
 * of rho kept (FP32).  Equal significances go to the lowest template id. */
typedef struct {
  uint32_t segment;
  uint32_t lag;
  uint32_t template_id;
  float snr;
} bfs_peak;

/* One coincidence of a detector pair (24 bytes): at lag `lag` both channels of
 * pair `pair` carry a per-lag max-projected hit and the initial frequencies of
 * the two winning templates differ by less than the plan's coinc_delta_hz
 * (the simultaneous hits with close frequency pairs of Sec. 5 and Table 3).
 * snr_a / snr_b: rho / sigma of the winners in channels 2 pair and
 * 2 pair + 1 (FP32, sign kept). */
typedef struct {
  uint32_t pair;
  uint32_t lag;
  uint32_t template_a;
  uint32_t template_b;
  float snr_a;
  float snr_b;
} bfs_coinc;

/* Plan descriptor.  All pointers are host memory, read during the call only. */
typedef struct {
  uint32_t n;                   /* largest segment length N: power of two, supported
                                   2^10..2^17 (BFS_FP32*) or 2^10..2^14 (BFS_FP64) */
  uint32_t n_min;               /* smallest segment length (power of two <= n;
                                   0 = n).  The plan keeps one resident bank per
                                   power of two in [n_min, n] (each template
                                   zero-padded to that length), so segments of
                                   every such length can share a filter call */
  double fs;                    /* sample rate in Hz, > 0 */
  uint32_t n_f0, n_fdot;        /* grid size; K = n_f0 * n_fdot */
  double f0_lo, f0_hi;          /* initial frequency range (Hz), inclusive */
  double fdot_lo, fdot_hi;      /* frequency rate range (Hz/s), inclusive */
  uint32_t n_tau;               /* number of durations, >= 1 */
  const double* tau;            /* [n_tau] durations in s; template j uses tau[j % n_tau];
                                   every L = round(tau * fs) must be <= n_min */
  uint32_t taper;               /* 0: none, 1: symmetric Hann */
  const double* explicit_templates; /* optional host [n_explicit][explicit_len] FP64
                                       bank used as given (no normalisation);
                                       when set, the grid fields are ignored;
                                       explicit_len <= n_min */
  uint32_t n_explicit, explicit_len;
  double kappa;                 /* threshold multiple, >= 0 (0 keeps every nonzero lag) */
  bfs_precision precision;
  uint64_t tail_capacity;       /* device tail slots per job, >= 1 */
  uint64_t hbm_budget_bytes;    /* 0: the device's free memory.  Plan memory
                                   (banks, tables) and every live job's buffers
                                   count against it; a call that would exceed it
                                   fails with BFS_ERR_OUT_OF_MEMORY */
  int device;                   /* HIP device ordinal */
  uint32_t flags;               /* BFS_PLAN_* bits, 0 for none */
  uint32_t candidate;           /* 0: the default kernel (or the autotuned
                                   one); i > 0: candidate i - 1 at every length
                                   that has that many (manual tuning, tests) */
  uint32_t tile;                /* 0: the default (or autotuned) segment tile;
                                   t > 0: t segments per tile at every length */
  double kappa_hi;              /* 0: tails are |rho| > kappa sigma; > kappa: a
                                   finite band kappa sigma < |rho| < kappa_hi sigma
                                   (the deep-search generalisation of Eq. 9 the
                                   paper proposes in Sec. 5) */
  double coinc_delta_hz;        /* 0: none; > 0 (BFS_PLAN_PAIRS | BFS_PLAN_PROJECT
                                   grid plans only): after the projection, every
                                   lag where both channels of a pair have a hit
                                   whose winning templates' initial frequencies
                                   differ by less than this is listed as a
                                   coincidence (Delta = 50 Hz in Sec. 5) */
} bfs_plan_desc;

/* Read-only facts about a plan. */
typedef struct {
  uint32_t n, m, k;             /* largest N, N/2, number of templates */
  uint32_t threads_per_correlation; /* workgroup size of the fused kernel at N */
  uint64_t bank_bytes;          /* resident template spectra, all lengths */
  uint64_t plan_bytes;          /* all device memory held by the plan */
  uint32_t precision;
  uint32_t n_min;               /* smallest accepted segment length */
  uint64_t held_bytes;          /* device bytes the plan holds now: plan memory,
                                   live jobs' buffers and released buffer sets kept
                                   for reuse; never above the HBM budget */
} bfs_plan_info;

/* The fused kernel a plan runs at one segment length. */
typedef struct {
  uint32_t n;                   /* segment length */
  uint32_t r1, r2, r3;          /* radices of the on-chip transform (length r1*r2*r3) */
  uint32_t threads;             /* workgroup size (one correlation per workgroup) */
  uint32_t load_group;          /* spectrum elements loaded ahead per group */
  uint32_t split;               /* 1: the length-n/2 inverse transform runs as two halves */
  uint32_t candidate;           /* index of the chosen candidate */
  uint32_t n_candidates;        /* candidates built for this length */
  float tuned_us[8];            /* per candidate: measured microseconds per
                                   correlation (BFS_PLAN_AUTOTUNE), else 0 */
  uint32_t tile;                /* segments per tile of the workgroup order: the
                                   workgroups of one template and `tile` segments
                                   run back to back on one XCD, which serves the
                                   template's spectrum from its L2 */
  float tile_us[5];             /* measured microseconds per correlation for tiles
                                   1, 2, 4, 8, 16 on 16 segments (BFS_PLAN_AUTOTUNE),
                                   else 0 */
  uint32_t fused;               /* 1: templates synthesised per correlation (no bank) */
  uint32_t fused_rows;          /* fused: nonzero input rows of the forward
                                   transform's first pass */
  uint32_t loop;                /* 1: as many workgroups as the device holds at
                                   once, each looping over correlations */
} bfs_kernel_info;

/* Build a plan: synthesises every template on the device (FP64 phase and
 * norm), transforms it (real FFT of the template zero-padded to each
 * accepted length, Sec. 3.2 step (ii)) and keeps the spectra resident in
 * HBM.  On error *out is NULL and nothing stays allocated. */
bfs_status bfsearch_plan(const bfs_plan_desc* desc, bfs_plan** out);

/* Queue the hot path for n_segments segments on hip_stream (a hipStream_t;
 * NULL = the null stream) and return at once.
 *   y_dev: caller-owned device memory holding the samples; double for
 *          BFS_FP64 plans, float otherwise.  It must stay valid until the
 *          job's kernels have finished (fetch, timing or release).
 *   seg_lengths: host [n_segments], each a power of two in [n_min, n]; NULL
 *          means every segment has length n.
 *   seg_offsets: host [n_segments], element offset of each segment from
 *          y_dev; NULL means the segments are packed back to back in order.
 *   n_segments: 1..65535 (BFS_PLAN_PAIRS: even, the two channels of each
 *          pair of equal length, else BFS_ERR_INVALID_ARG).
 * Segments of one length form a group.  Per group: forward real FFT of each
 * segment (Eq. 5); then one fused kernel per (template, segment) computes
 * C = conj(W) Y, sigma by Parseval in FP64 (Eq. 7), the inverse FFT on chip
 * (Eq. 5), the threshold (Eq. 9) and wave-ballot compaction of the tails into
 * the job's device buffer.  Segment ids in tails and sigma are the indices
 * into the caller's arrays.  The segment table is read before return.
 * Streams: the job starts after the work queued on hip_stream before the
 * call.  Outside BFS_PLAN_GRAPH plans, the segment transforms run on
 * hip_stream and the fused kernels on an internal stream of the plan paired
 * with hip_stream (created on first use, at most 16 per plan with later
 * caller streams sharing them, destroyed with the plan), queued
 * after those transforms; so the next call's transforms overlap this call's
 * correlations, and work queued later on hip_stream is ordered after the
 * transforms only.  BFS_PLAN_GRAPH plans replay the whole job on hip_stream.
 * Wait for the job through the job calls (fetch, poll, timing, release), or a
 * device-wide synchronisation. */
bfs_status bfsearch_filter(bfs_plan* plan, const void* y_dev, const uint64_t* seg_offsets,
                           const uint32_t* seg_lengths, uint32_t n_segments, void* hip_stream,
                           bfs_job** out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the hot
 * path of bfsearch_filter with no allocation and no host synchronisation.
 * It makes no hipMalloc, hipFree or allocating library call; the segment
 * spectra live in a fixed scratch area of the library, 16 MiB per device
 * (BFS_NOALLOC_SCRATCH_BYTES), held from the first plan on that device until
 * the process ends.  Queued on hip_stream (NULL = the null stream); returns
 * at once.
 *   y_dev: n_segments segments of seg_len samples (0 = the plan's largest
 *          length; an accepted length) packed back to back, float (double for
 *          BFS_FP64 plans), caller device memory.
 *   tails_dev: caller device memory for tail_capacity records of the
 *          plan's type: bfs_tail (16 bytes) for BFS_FP32* plans, bfs_tail64
 *          (24 bytes) for BFS_FP64 plans; unsorted, in the order the kernels
 *          reserve them; tails past tail_capacity are counted, not written.
 *   count_dev: caller device memory, one uint64_t: set to 0 on the stream,
 *          then to the exact number of tails found.
 *   sigma_dev: caller device memory [n_segments][K] doubles, or NULL.
 * The spectra need n_segments * seg_len * 4 bytes (FP32; FP64: 8), twice that
 * for lengths of 2^12 samples and more and for fused plans (a scratch of the
 * same size for the segment transform or the fused layout); more than the
 * scratch area is BFS_ERR_SCRATCH_LIMIT, before anything is queued.
 * BFS_ERR_INVALID_ARG for projection plans, an odd count on pair plans, or
 * a length the plan does not hold.  Every call on one device shares its
 * scratch area, so calls whose work overlaps on the device (different
 * streams without ordering between them) race and give wrong results; calls
 * queued on one stream are ordered and safe.  Plans on other devices have
 * their own area. */
#define BFS_NOALLOC_SCRATCH_BYTES (16u << 20)
bfs_status bfsearch_filter_noalloc(bfs_plan* plan, const void* y_dev, uint32_t seg_len, uint32_t n_segments,
                                   void* tails_dev, uint64_t tail_capacity, uint64_t* count_dev, double* sigma_dev,
                                   void* hip_stream);

/* Gather the tails to the host (Sec. 3.3: only the hits above threshold
 * cross to the host, never the correlation output itself; this is the
 * paper's mode that gathers every hit, without max selection).  Waits for
 * the job, copies its tails to out_host sorted by (segment, template_id,
 * lag), and reports counts.
 *   capacity: slots in out_host; *n_written <= capacity; *n_total = exact
 *   number of tails the kernels found.  Returns BFS_ERR_TAIL_OVERFLOW when
 *   *n_total exceeds capacity or the plan's tail_capacity; the records then
 *   written are an arbitrary subset. */
bfs_status bfsearch_fetch_tails(bfs_job* job, bfs_tail* out_host, uint64_t capacity,
                                uint64_t* n_written, uint64_t* n_total);

/* As bfsearch_fetch_tails, into 24-byte records with an FP64 rho (exact for
 * FP64 plans, the FP32 value widened for the others). */
bfs_status bfsearch_fetch_tails64(bfs_job* job, bfs_tail64* out_host, uint64_t capacity,
                                  uint64_t* n_written, uint64_t* n_total);

/* BFS_PLAN_PROJECT plans: wait for the job and copy its per-lag max
 * projection to out_host, sorted by (segment, lag), one entry per lag that
 * carries at least one tail (the paper's array A reduced over templates, with
 * the data of maximal rho per offset as in its host array B, Sec. 3.3).  The
 * kernels raise each lag's entry with a 64-bit atomicMax of
 * (significance bits, lowest template id, sign), so the result is the same
 * whatever the order of the updates.  *n_total = entries found; returns
 * BFS_ERR_TAIL_OVERFLOW when it exceeds capacity (the first `capacity` in
 * order are written).  BFS_ERR_INVALID_ARG for plans without the flag;
 * bfsearch_fetch_tails likewise refuses projection plans. */
bfs_status bfsearch_fetch_projection(bfs_job* job, bfs_peak* out_host, uint64_t capacity,
                                     uint64_t* n_written, uint64_t* n_total);

/* Plans with coinc_delta_hz > 0: wait for the job and copy its coincidences
 * (Sec. 5, Table 3: simultaneous hits of the two channels of a pair with
 * close template frequencies) to out_host sorted by (pair, lag).  The device
 * finds them from the per-lag projections of both channels, comparing the
 * winners' initial frequencies in FP64.  *n_total = coincidences found;
 * BFS_ERR_TAIL_OVERFLOW when it exceeds capacity (the first `capacity` in
 * order are written).  BFS_ERR_INVALID_ARG for plans without a window. */
bfs_status bfsearch_fetch_coincidences(bfs_job* job, bfs_coinc* out_host, uint64_t capacity,
                                       uint64_t* n_written, uint64_t* n_total);

/* Wait for the job and copy sigma[s][j] (FP64, Eq. 6 by Parseval) to out_host
 * ([n_segments][K] doubles). */
bfs_status bfsearch_fetch_sigma(bfs_job* job, double* out_host);

/* Device time of the job's kernels in milliseconds, measured with HIP events
 * on the streams the kernels run on: *corr_ms from the start of the first fused
 * correlation kernel to the end of the last (events recorded by those launches
 * themselves; the whole replayed graph for BFS_PLAN_GRAPH plans), *total_ms the
 * whole job.  Waits for the job. */
bfs_status bfsearch_job_timing(bfs_job* job, float* corr_ms, float* total_ms);

/* Non-blocking completion check: *done = 1 once every kernel of the job has
 * finished, else 0. */
bfs_status bfsearch_job_poll(bfs_job* job, int* done);

/* Device bytes a filter call with these segment lengths (NULL = all n) takes
 * from the plan's HBM budget while its job is live (segment spectra,
 * transform scratch, sigma, tail buffer, segment table).  No device access;
 * lets a scheduler admit work by budget before calling bfsearch_filter. */
bfs_status bfsearch_plan_job_bytes(const bfs_plan* plan, const uint32_t* seg_lengths, uint32_t n_segments,
                                   uint64_t* bytes);

/* Return the job's buffers to the plan.  The job pointer is invalid after. */
bfs_status bfsearch_job_release(bfs_job* job);

/* Free a plan.  All its jobs must have been released. */
bfs_status bfsearch_destroy(bfs_plan* plan);

bfs_status bfsearch_plan_get_info(const bfs_plan* plan, bfs_plan_info* out);

/* The kernel configuration the plan uses at segment length n (0 = the
 * largest); BFS_ERR_INVALID_ARG for a length the plan does not hold. */
bfs_status bfsearch_plan_kernel_info(const bfs_plan* plan, uint32_t n, bfs_kernel_info* out);

/* Diagnostic: the same fused kernel, writing every rho value instead of
 * compacting tails, for n_segments segments of length seg_len (0 = n)
 * packed back to back at y_dev.  rho_dev: caller device memory
 * [n_segments][K][seg_len] of the plan's sample type (double or float);
 * sigma_dev: [n_segments][K] doubles (may be NULL).  Returns after the
 * kernels finish. */
bfs_status bfsearch_correlate_dense(bfs_plan* plan, const void* y_dev, uint32_t seg_len, uint32_t n_segments,
                                    void* rho_dev, double* sigma_dev, void* hip_stream);

/* Diagnostic: as bfsearch_correlate_dense for the templates first..first+count-1
 * only (the parity checks of large banks take them block by block).
 * rho_dev: [n_segments][count][seg_len] of the plan's sample type;
 * sigma_dev: [n_segments][count] doubles (may be NULL).  BFS_ERR_INVALID_ARG
 * when the range leaves the bank or count is 0.  Returns after the kernels
 * finish. */
bfs_status bfsearch_correlate_dense_range(bfs_plan* plan, const void* y_dev, uint32_t seg_len, uint32_t n_segments,
                                          uint32_t first, uint32_t count, void* rho_dev, double* sigma_dev,
                                          void* hip_stream);

/* Diagnostic: template spectra W_j[k], k = 0..n/2, at segment length n (0 =
 * the plan's largest), as interleaved FP64 complex into caller device memory
 * out_dev [count][n/2 + 1][2], for templates first..first+count-1.  Queued on
 * hip_stream. */
bfs_status bfsearch_plan_spectra(const bfs_plan* plan, uint32_t n, uint32_t first, uint32_t count,
                                 double* out_dev, void* hip_stream);

/* Diagnostic: the job's segment spectra Y_s[k], k = 0..N_s/2, as interleaved
 * FP64 complex into out_dev, segment after segment in the caller's order
 * (segment s starts sum_{s' < s} (N_s'/2 + 1) complex values in).  Queued on
 * the job's stream. */
bfs_status bfsearch_job_spectra(const bfs_job* job, double* out_dev);

const char* bfsearch_status_string(bfs_status s);

#ifdef __cplusplus
}
#endif

#endif /* BFSEARCH_H */
