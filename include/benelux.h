/*
 * benelux.h -- C-ABI of the MI355X (gfx950) Benelux-pair search library.
 *
 * What it computes (Hercher, "On one of Erdos' Problems -- An Efficient Search
 * for Benelux Pairs", arXiv:2506.01099):
 *   rad(n)      product of the distinct primes dividing n, rad(1) = 1
 *               (Section 2.1, definition of the radical; computed by the sieve
 *               of Algorithm 1).
 *   S_x         the set {rad(x), rad(x+1)} (Section 2.1, before Algorithm 2).
 *   pair (m,n)  m < n with S_m = S_n.  First kind: rad(m) = rad(n) and
 *               rad(m+1) = rad(n+1); second kind: rad(m) = rad(n+1) and
 *               rad(m+1) = rad(n) (Section 1).  A collision is of the first kind
 *               when rad(m) = rad(n), else of the second (Algorithm 2).
 *               Every pair inside a group of equal sets is reported, as the
 *               probe chains of Algorithm 3 do.
 *
 * Conventions shared by every entry point:
 *   - Return value: BX_OK (0) on success, a negative BX_E* code on failure; the
 *     message of the last failure on the calling thread is bx_last_error().
 *   - Integers are unsigned 64-bit.  Every value whose radical is needed must be
 *     below BX_VALUE_LIMIT (2^42) and at most the context's hi_max.
 *   - Pair lists are malloc'd by the library, sorted by (query, m, n), and
 *     released by the caller with bx_free().  An empty result is count 0 and a
 *     NULL list.
 *   - Calls on one context are serialised by the library (one at a time); use
 *     one context per host thread for concurrency.
 *   - All device work runs on the context's HIP stream (bx_set_stream); every
 *     blocking call returns after that stream has drained.
 */
#ifndef BENELUX_H
#define BENELUX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BX_VALUE_LIMIT (1ull << 42)

/* kinds: a bit mask.  BX_THIRD adds Erdős's third condition (the problem in
 * the paper's abstract and introduction): a first-kind pair with also
 * rad(m+2) = rad(n+2) is reported with kind = 1 | BX_THIRD = 5.  kinds =
 * BX_THIRD alone reports only such pairs; it needs b + 1 <= hi_max. */
enum { BX_FIRST = 1, BX_SECOND = 2, BX_BOTH = 3, BX_THIRD = 4 };

enum {
  BX_OK = 0,
  BX_EINVAL = -1,    /* bad argument: lo = 0, hi < lo, kinds not in 1..7, NULL pointer  */
  BX_ERANGE = -2,    /* a value needs a radical beyond hi_max or BX_VALUE_LIMIT         */
  BX_ENOMEM = -3,    /* host or device allocation failed, or the HBM budget is too small */
  BX_EDEVICE = -4,   /* a HIP runtime error; the message names it                       */
  BX_EBUSY = -5,     /* serving: request beyond the budget, or not admissible at once
                        with option submit_wait = 0; bx_take of an unfinished request */
  BX_EINTERNAL = -6  /* a device-side consistency check failed (see bx_last_error)     */
};

/* One reported pair.  kind is 1 or 2, or 5 (first kind and third condition)
 * when BX_THIRD is asked for; query is the index of the range query it
 * belongs to (0 for single-range calls). */
typedef struct {
  uint64_t m;
  uint64_t n;
  uint32_t kind;
  uint32_t query;
} bx_pair;

typedef struct bx_ctx bx_ctx;

/* Create a context on HIP device `device` able to sieve values up to hi_max
 * (< 2^42).  It builds the prime tables (all primes <= sqrt(hi_max), and every
 * odd prime power p^k <= hi_max with k >= 2; the "list of primes sent to the
 * GPU once" of Section 3.1) and keeps them resident in device memory.
 * hbm_budget_bytes bounds the device workspace (0 = 85% of free memory).
 * Errors: BX_EINVAL (NULL ctx), BX_ERANGE (hi_max too large), BX_EDEVICE,
 * BX_ENOMEM. */
int bx_create(bx_ctx** ctx, int device, uint64_t hi_max, uint64_t hbm_budget_bytes);
void bx_destroy(bx_ctx* ctx);

/* Use `hip_stream` (a hipStream_t, e.g. torch's current stream) for all later
 * device work of this context; NULL restores the context's own stream.  The
 * caller keeps ownership of the stream. */
int bx_set_stream(bx_ctx* ctx, void* hip_stream);

/* rad(x) for x in [lo, hi) into the caller-owned host buffer out[hi - lo]
 * (Algorithm 1 over the interval [start, start + length[ ).  lo >= 1, hi >= lo,
 * hi <= hi_max.  Empty when hi == lo. */
int bx_radical_segment(bx_ctx* ctx, uint64_t lo, uint64_t hi, uint64_t* out);

/* Same, writing into caller-owned device memory dev_out[hi - lo] on the HIP
 * stream `hip_stream`, which is the caller's: NULL is HIP's default (null)
 * stream, as in HIP's own calls (and PyTorch's default stream), not the
 * context's stream.  The kernels are ordered after the context's earlier work.
 * Returns once they are queued; the caller synchronises the stream. */
int bx_radical_segment_dev(bx_ctx* ctx, uint64_t lo, uint64_t hi, uint64_t* dev_out, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * bx_radical_segment_dev without any allocation.  Its kernels keep their
 * scratch (counter words, the query table, the sparse-hit spill of at most
 * 512 sieve workgroups x 4096 hits) in one fixed device array of about 16 MB
 * that the library holds on every device it runs on until the process ends;
 * nothing is allocated or freed by the call (the context's prime tables come
 * from bx_create).  Arguments, layout and ownership as bx_radical_segment_dev.
 * Unlike it, the call returns after its kernels have finished (it reads back
 * the overflow word).  Errors: those of bx_radical_segment_dev; BX_ENOMEM
 * before any launch when the context's segment length would need more than
 * half the scratch's sparse-hit room on average (at most 2^19 with the 8192
 * tile, 2^18 with the 2048 tile), and BX_ENOMEM after the launch if a segment
 * overflowed it anyway (dev_out is then incomplete).  Calls on one device share
 * its scratch and keep the last call's contents; the library serialises them
 * (a per-device lock held until the kernels have finished), so they do not
 * race, but they do not overlap either. */
int bx_radical_segment_dev_noalloc(bx_ctx* ctx, uint64_t lo, uint64_t hi, uint64_t* dev_out, void* hip_stream);

/* All pairs 1 <= m < n <= N whose kind is in `kinds` (Algorithm 2's output,
 * found by the hash-partitioned join); radicals are sieved over [1, N + 1].
 * *out is malloc'd, *count set.  N + 1 <= hi_max. */
int bx_benelux_search(bx_ctx* ctx, uint64_t N, uint32_t kinds, bx_pair** out, size_t* count);

/* Range form: pairs with max(a,1) <= m < n < b (radicals over [max(a,1), b]),
 * both members inside the range: Algorithm 3 reports the pairs whose larger
 * member lies in the chunk it holds, Algorithm 1 sieves an interval
 * [start, start + length[, and this call does both for one interval.
 * bx_benelux_search(N) equals bx_search_range(1, N + 1).  b <= hi_max.
 * Errors: BX_EINVAL (NULL pointer, kinds not in 1..7), BX_ERANGE (b beyond
 * hi_max), BX_ENOMEM, BX_EDEVICE, BX_EINTERNAL.  a = 0 is read as 1; fewer
 * than two integers give no pair. */
int bx_search_range(bx_ctx* ctx, uint64_t a, uint64_t b, uint32_t kinds, bx_pair** out, size_t* count);

/* Batched range queries: for each i < q, the pairs inside [a[i], b[i]) (each
 * query is joined only with itself).  One pipeline serves all queries, captured
 * in a HIP graph.  b[i] - a[i] <= 2^28 each, q <= 32768.  *out is malloc'd and
 * holds the pairs of query i at [offsets[i], offsets[i+1]); offsets is
 * caller-owned with q + 1 entries. */
int bx_search_batch(bx_ctx* ctx, const uint64_t* a, const uint64_t* b, size_t q, uint32_t kinds, bx_pair** out,
                    size_t* offsets);

/* Serving (continuous batching of range requests, each over an interval
 * [start, start + length[ as in Algorithm 1, arriving over time).  bx_serve_start starts max_inflight lanes (1..8), each a context of
 * its own with its own stream and workspace and one scheduler thread; a lane
 * takes the owner's search options (tile, sieve, seg_len, prune, join,
 * fp_bits, third_offset, group) as they are when serving starts.  A free lane
 * admits queued requests in arrival order into one batch while the device
 * bytes of all lanes' workspaces -- this lane's grown to what the batch's plan
 * needs -- stay within budget_bytes (0 = half the owner's budget); a lane that
 * finds no room lets its own idle workspace go.  Batches of different lanes
 * overlap on the device.  bx_submit never blocks.  With the owner's option
 * "submit_wait" = 1 (default) it queues the request and returns BX_EBUSY only
 * when the request alone needs more than the budget; with "submit_wait" = 0
 * it also returns BX_EBUSY, queueing nothing, unless the request can be
 * admitted at once (no request queued, and an idle lane whose workspace for
 * this request alone fits beside the other lanes').  bx_poll reports
 * completion; bx_take hands over the pair list (malloc'd, sorted by (m, n))
 * and releases the ticket (BX_EBUSY while the request runs); bx_take_timed
 * also gives the submit and completion times, in seconds on the library's
 * monotonic clock (bx_now; either pointer may be NULL). */
int bx_serve_start(bx_ctx* ctx, uint64_t budget_bytes, int max_inflight);
int bx_serve_stop(bx_ctx* ctx);
int bx_submit(bx_ctx* ctx, uint64_t a, uint64_t b, uint32_t kinds, uint64_t* ticket);
int bx_poll(bx_ctx* ctx, uint64_t ticket, int* done);
int bx_take(bx_ctx* ctx, uint64_t ticket, bx_pair** out, size_t* count);
int bx_take_timed(bx_ctx* ctx, uint64_t ticket, bx_pair** out, size_t* count, double* t_submit, double* t_done);

/* Admission record of the running server. */
typedef struct {
  uint64_t budget_bytes;  /* the admission budget                                         */
  uint64_t peak_bytes;    /* largest sum of the lanes' workspaces, reserved or held       */
  uint64_t held_bytes;    /* that sum now                                                 */
  uint64_t admitted;      /* requests admitted so far                                     */
  uint64_t batches;       /* batches they ran in                                          */
  uint32_t max_batch;     /* most requests in one batch                                   */
  uint32_t lanes;
  uint64_t memory_waits;  /* times a free lane found queued requests but no room          */
  uint64_t releases;      /* times a lane let its workspace go to make room               */
} bx_serve_info;
int bx_serve_get_info(bx_ctx* ctx, bx_serve_info* out);
double bx_now(void);

/* Autotuner.  Times the batched search of the queries [a[i], b[i]) (q >= 1;
 * one query [1, N+1) stands for a plain search) under every combination of
 * sieve tile {2048, 8192}, segment length {2^15 .. 2^19} and second-level group
 * {2, 4, 8}, then, with the fastest of those, every small-query cutoff
 * {0, 1024, 2048, 4096, 8192} and workgroup size {256, 512, 1024} of that
 * class; `reps` timed runs per setting after one warm-up.  Keeps the fastest,
 * applies it to ctx and, when path is not NULL, writes it as a one-line JSON
 * object (arch, tile, seg_len, group, small_max, small_block, ms).  Results of
 * every run are checked
 * to be identical.  Errors as bx_search_batch, plus BX_EDEVICE when a file
 * cannot be written and BX_EINTERNAL when two settings disagree. */
int bx_autotune(bx_ctx* ctx, const uint64_t* a, const uint64_t* b, size_t q, int reps, const char* path);
/* Apply a tuning file written by bx_autotune; a file for another GPU
 * architecture is ignored (returns BX_OK, nothing changes). */
int bx_load_tuning(bx_ctx* ctx, const char* path);

/* Statistics of the last completed call on this context (device times from HIP
 * events recorded on the stream the kernels ran on). */
typedef struct {
  uint32_t passes;            /* hash passes run (including split re-runs)        */
  uint32_t retries;           /* passes re-run split in two after an overflow     */
  uint64_t integers;          /* x values whose keys were generated, per pass     */
  uint64_t entries;           /* entries written by all passes                    */
  uint64_t candidates;        /* candidate pairs emitted by the join              */
  uint64_t pairs;             /* verified pairs reported (kinds filter applied)   */
  uint32_t launches[6];       /* launches per kernel: sieve, partition, join, verify, radicals, small */
  double kernel_ms[6];        /* summed device time per kernel, same order        */
  double total_ms;            /* host wall time of the call                       */
  uint32_t b1_bits, b2_bits;  /* partition fan-outs used                          */
  uint32_t seg_len, tile;     /* segment length and LDS tile used by the sieve    */
  double graph_ms;            /* device time of the captured graph (batched calls) */
  uint64_t joined;            /* entries the join kernels read (equals entries)   */
  uint64_t false_candidates;  /* candidates whose sets differ (dropped by verify) */
  uint32_t l2_entry_bytes;    /* bytes per second-level entry: 8 (compact words) or 12 */
  uint32_t word_matches;      /* compact words whose kept bits met (each pair read back
                                 from the first level; candidates are those of them
                                 with equal whole fingerprints and queries)        */
} bx_stats;
int bx_get_stats(bx_ctx* ctx, bx_stats* out);

/* Options (name = value); unknown names are BX_EINVAL.
 *   "passes"       force the number of hash passes (any count, 0 = plan)
 *   "seg_len"      sieve segment length (multiple of the tile, 0 = default)
 *   "timing"       1 = record HIP events per kernel (default 1)
 *   "b1_bits"      force the first partition fan-out (0 = plan)
 *   "b2_bits"      force the second partition fan-out, <= 11 (0 = plan)
 *   "group"        first-level buckets per second-level launch (1, 2, 4, 8; 0 = 8)
 *   "tile"         sieve LDS tile: 2048 (two workgroups per CU) or 8192 (one; 0 = 8192)
 *   "graph"        1 = batched calls run as one captured HIP graph (default 1)
 *   "fp_bits"      for tests of the verification: keep only the top 11 and
 *                  the low fp_bits bits of the 53-bit fingerprints (v in
 *                  [12, 53]; 0 = all), so that different sets collide and
 *                  must be dropped by the verification
 *   "join"         0 = LDS hash join per partition (default), 1 = sort join per
 *                  partition (Algorithm 2 on each partition, every pair of a
 *                  run of equal keys reported; an ablation)
 *   "third_offset" for tests of the third condition: compare rad(m + d) and
 *                  rad(n + d) with d = value (in [0, 64]) instead of d = 2,
 *                  so that kinds bit BX_THIRD marks known pairs (d = 0 or 1
 *                  marks every first-kind pair; default 2)
 *   "prune"        1 = only integers that can be a member of a pair enter the
 *                  join (default 1; the pair lists are the same either way:
 *                  a pair's larger member n has n and n+1 non-squarefree, and
 *                  a squarefree smaller member m has n or n+1 = m*t with
 *                  t >= max(2, rad(m+1) - 1), likewise for m+1)
 *   "small_max"    queries of 2 .. small_max integers (at most 8192; 0 = none)
 *                  are each sieved, member-tested and hash-joined by one
 *                  workgroup in LDS, with no entry written to device memory
 *                  and no partition or join launch (default 8192; the pairs
 *                  are the same either way)
 *   "small_block"  threads per workgroup of that class: 256, 512 or 1024
 *                  (0 = 1024)
 *   "submit_wait"  serving: 1 = bx_submit queues (default), 0 = bx_submit
 *                  refuses with BX_EBUSY what cannot be admitted at once
 *   "compact"      the second partition level stores 8-byte words (the
 *                  entry's index among its first-level bucket's regions and
 *                  the low fingerprint bits; the partition index stands for
 *                  the top bits) instead of 12-byte entries where the plan
 *                  allows it: full fingerprints, hash join, and at most 3e5
 *                  expected random matches of the kept bits (the join reads
 *                  both entries of a match back from the first level).
 *                  0 = never, 1 = where the plan allows (default)
 *   "compact_fp_bits" for tests of the compact join: keep only this many low
 *                  fingerprint bits in a compact word (12 .. 40; 0 = all the
 *                  word holds), so that different sets meet
 *   "schedule"     single-range searches (bx_benelux_search, bx_search_range):
 *                  0 = hash-partitioned passes (default); 1 = Algorithm 3's
 *                  schedule (chunks of s values overlapping by one, each
 *                  inserted into an open-addressing table of 4s slots in device
 *                  memory, every earlier chunk sieved again and probed); 2 =
 *                  Algorithm 2 (the list of (S_n, n) over the whole range,
 *                  radix-sorted by a fingerprint of S_n, every pair inside a
 *                  run of equal keys verified; 32 bytes of device memory per
 *                  kept integer, BX_ENOMEM beyond the budget).  Same pair lists;
 *                  baselines of the paper's own designs.  Batched calls and
 *                  serving always use 0.
 *   "a3_chunk_log2" log2 of Algorithm 3's chunk size s (10 .. 27; 0 = 27)  */
int bx_set_option(bx_ctx* ctx, const char* name, int64_t value);

void bx_free(void* p);
const char* bx_last_error(void);

/* Thin wrappers over a lazily created default context on device 0 with
 * hi_max = 2^42 - 1 (the two calls of the method's boundary). */
int benelux_search(uint64_t N, uint32_t kinds, bx_pair** out, size_t* count);
int radical_segment(uint64_t lo, uint64_t hi, uint64_t* out);

#ifdef __cplusplus
}
#endif
#endif /* BENELUX_H */
