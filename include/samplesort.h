/*
 * samplesort.h -- C ABI of the MI355X (gfx950) oversampling sample sort.
 *
 * The method (Gerbessiotis, arXiv 1608.08648): draw a sample of the keys
 * (random oversampling, Alg. 2 step 2, or deterministic regular
 * oversampling, Alg. 1 steps 1-2), sort it, take p-1 equidistant splitters
 * (step 3), split every key into one of p buckets (step 4; ties between
 * equal keys broken by input position, Section 2.2), and sort every bucket
 * on its own so the buckets concatenate into the output (Section 1).  Here
 * sampling precedes the split (the traditional organisation described in
 * Section 1 and after Claim 1) and every step runs in HIP kernels on one
 * GPU.
 *
 * Conventions shared by every entry point:
 *  - All array arguments are DEVICE pointers unless stated otherwise.  The
 *    caller owns every buffer, including the workspace `ws`; no entry point
 *    allocates device memory, so calls may be captured into a HIP graph.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    work is enqueued on it; the calls return before the GPU finishes.
 *  - The return value covers argument checks and launch errors only:
 *    SS_OK (0) or a negative SS_E* code, with a message in ss_last_error().
 *    Conditions detected on the device are reported by ss_status().
 *  - In-place use is allowed (keys_in == keys_out, vals_in == vals_out);
 *    partial overlap of an input with an output is rejected (SS_EINVAL).
 *  - The result is always the stable order: equal keys keep their input
 *    order (Section 1's definition).  `stable = 0` is accepted and gives the
 *    same result.
 *  - Keys order as integers (unsigned or two's complement) or, for floats,
 *    by IEEE 754 totalOrder (-NaN < -inf < ... < -0 < +0 < ... < +inf < +NaN).
 */
#ifndef SAMPLESORT_H
#define SAMPLESORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* key types */
enum { SS_U32 = 0, SS_I32 = 1, SS_F32 = 2, SS_U64 = 3, SS_I64 = 4, SS_F64 = 5 };

/* payload types: a payload is moved bit-exactly with its key.
 * SS_V_IOTA32 / SS_V_IOTA64: no payload is read (vals_in must be NULL); the
 * payload of each key is its index within its array or segment, written as
 * uint32 / int64, i.e. the stable sorting permutation.  SS_V_IOTA64 is
 * sorted as a 32-bit index in the workspace (4 bytes per element more) and
 * widened into vals_out at the end; vals_out outside a segmented sort's
 * [offsets[0], offsets[num_segments]) is not written. */
enum { SS_V_NONE = 0, SS_V_B32 = 1, SS_V_B64 = 2, SS_V_IOTA32 = 3, SS_V_IOTA64 = 4 };

/* sampling rule */
enum { SS_RANDOM = 0,   /* Alg. 2: p*s-1 keys drawn uniformly (with replacement) */
       SS_REGULAR = 1   /* Alg. 1: p blocks, s*p evenly spaced keys per sorted block */ };

/* flags */
#define SS_F_EXPORT_STAGES  1u  /* keep the top-level sample, splitters and bucket counts in ws */
#define SS_F_FORCE_PIPELINE 2u  /* run the sampling pipeline even when n fits one work-group */
#define SS_F_NO_RECURSION   4u  /* plan no split level below the top one: a bucket too large for
                                   one work-group is then sorted by a one-work-group merge sort
                                   (slow; for tests of that path) */
#define SS_F_NO_WIDE        8u  /* keys-only sorts of 4-byte keys with p >= 1024 move the keys in
                                   two passes (64 coarse buckets, then p/64 fine ones); this flag
                                   keeps the one-pass split instead (for comparisons) */
#define SS_F_SORT_FIRST    16u  /* the organisation Alg. 1 and Alg. 2 state: sort the p blocks
                                   first (step 1), place the splitters in each sorted block by
                                   binary search (step 4), and form bucket j from the p runs the
                                   splitters cut out of the blocks (step 5).  Every key type and
                                   payload; single arrays only (SS_EINVAL for the segmented
                                   sort); p at most SS_P_MAX; no level below.  Without the flag
                                   the keys are classified and moved unsorted (the split-first
                                   organisation, the default). */
#define SS_F_SF_MERGE      32u  /* with SS_F_SORT_FIRST: step 5 merges each bucket's p runs (the
                                   paper's merging, lg p pairwise rounds in LDS) instead of
                                   gathering them and sorting the bucket.  4-byte keys without
                                   payload only (SS_EINVAL otherwise). */

/* return codes */
enum { SS_OK = 0, SS_EINVAL = -1, SS_EWORKSPACE = -2, SS_EHIP = -3, SS_EDEVICE = -4 };

/* Largest bucket count: the splitter search tree of one level lives in LDS. */
#define SS_P_MAX 4096u

/*
 * Parameters of the method.
 *  p        requested bucket count, a power of two in [2, SS_P_MAX].  The
 *           effective count is the largest power of two <= p that keeps the
 *           paper's preconditions: p <= n (Theorem 1), p*s < n/2 for random
 *           sampling (Claim 1), 4*s*p^2 <= n for regular sampling (the
 *           sample s*p^2 must be small against n, Theorem 1).
 *  s        oversampling factor as the paper states it per rule: RANDOM
 *           samples p*s-1 keys and takes every s-th as a splitter (Alg. 2);
 *           REGULAR takes s*p keys from each of the p sorted blocks (the
 *           paper's r = s, per-block sample r*p, Alg. 1) and every (s*p)-th
 *           of the s*p^2 samples as a splitter.  s >= 1.
 *  sampling SS_RANDOM or SS_REGULAR (applies to the top level; buckets too
 *           large for one work-group are split again with random sampling).
 *  stable   accepted for interface compatibility; the result is always stable.
 *  seed     seed of the counter-based generator (SplitMix64) behind random
 *           sampling; the same seed gives the same sample.
 *  flags    SS_F_* bits.
 *  tile     keys per work-group in the split passes (0 = chosen per p).
 * Every entry point that takes `const ss_params *prm` accepts NULL: the
 * tuned parameters of the call's size class (ss_get_tuning).
 */
typedef struct ss_params {
    uint32_t p;
    uint32_t s;
    int32_t sampling;
    int32_t stable;
    uint64_t seed;
    uint32_t flags;
    uint32_t tile;
} ss_params;

/* Where the top-level stages sit inside the workspace after a call with
 * SS_F_EXPORT_STAGES (byte offsets from ws; counts in elements).
 *  sample_ord / sample_tag : uint64[m]  sorted sample; ord = the key's
 *                            order-preserving unsigned image, tag = input index
 *  spl_ord / spl_tag       : uint64[p_eff-1] splitters (same encoding)
 *  counts                  : uint64[p_eff]  keys per bucket
 * p_eff == 1 means the call sorts directly with no sampling (n fits one
 * work-group, or no p >= 2 meets the preconditions). */
typedef struct ss_stage_info {
    uint32_t p_eff;
    uint32_t stride;      /* splitter i is the (i*stride)-th smallest sample */
    uint64_t m;           /* sample size */
    uint64_t sample_ord, sample_tag, spl_ord, spl_tag, counts;
    uint32_t direct;      /* 1 if no sampling pass runs */
    uint32_t levels;      /* split levels planned below the top one */
} ss_stage_info;

/* Last error message of the calling thread ("" if none).  Host only. */
const char *ss_last_error(void);

/* Workspace bytes a sample_sort_keys / sample_sort_pairs call with these
 * arguments needs.  Host only, no device call.  val_type = SS_V_NONE for a
 * keys-only sort. */
int ss_workspace_size(size_t n, int key_type, int val_type, const ss_params *prm, size_t *bytes_out);

/* Layout of the exported stages for the same arguments.  Host only. */
int ss_stage_layout(size_t n, int key_type, int val_type, const ss_params *prm, ss_stage_info *info);

/* Sort n keys ascending (stable).  keys_in/keys_out: device arrays of n keys
 * of key_type.  ws: device workspace of at least ss_workspace_size bytes,
 * 256-byte aligned; its contents on entry do not matter. */
int sample_sort_keys(const void *keys_in, void *keys_out, size_t n, int key_type,
                     const ss_params *prm, void *ws, size_t ws_bytes, void *stream);

/* Sort n (key, payload) pairs by key, stable; the payload follows its key.
 * vals_in: device array of n payloads of val_type (NULL for the IOTA types);
 * vals_out: device array of n payloads (uint32 for SS_V_B32/SS_V_IOTA32,
 * 8-byte for SS_V_B64/SS_V_IOTA64). */
int sample_sort_pairs(const void *keys_in, const void *vals_in, void *keys_out, void *vals_out,
                      size_t n, int key_type, int val_type, const ss_params *prm,
                      void *ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * keys-only sort of sample_sort_keys with its workspace in a static device
 * array of ss_noalloc_capacity_bytes() bytes (64 MiB) that the library holds
 * on every GPU it runs on until the process ends.  No device memory is
 * allocated and no workspace is passed.  A call whose plan needs more
 * scratch than the array holds (ss_workspace_size larger than the capacity:
 * about 2^22 4-byte keys with the tuned parameters) is refused with
 * SS_EWORKSPACE before anything is enqueued.  Every call on one GPU shares
 * that GPU's array, so calls that overlap in time on one GPU (other
 * streams, other host threads) race and must be serialised by the caller;
 * ss_status and ss_level_stats do not apply to it.  Arguments and results
 * are those of sample_sort_keys. */
int sample_sort_keys_noalloc(const void *keys_in, void *keys_out, size_t n, int key_type, const ss_params *prm,
                             void *stream);

/* Bytes of the static scratch array of sample_sort_keys_noalloc.  Host only. */
size_t ss_noalloc_capacity_bytes(void);

/* Fixed-width byte strings (the paper's measured keys, Section 3: random
 * 32-byte strings compared as memcmp does), sorted stably through their
 * index.  recs: device array of n strings of `width` bytes (a multiple of
 * 8 in [8, 256]), 8-byte aligned; perm_out: device int64[n], the stable
 * sorting permutation (string perm_out[i] is the i-th smallest, equal
 * strings in input order); recs_out: NULL, or a device array of n * width
 * bytes (8-byte aligned, not overlapping recs) that receives the sorted
 * strings.  The strings are not moved during the sort: their 64-bit
 * prefix words, read big-endian, travel with the index -- word 0 through
 * the pairs sort (sample, splitters, classification and buckets compare
 * the word), then, for runs of strings whose words so far are all equal,
 * the next word through the segmented sort, until no such run is left.
 * The call waits for `stream` once per round after the first (it reads
 * how many strings are still tied), so it cannot be captured into a HIP
 * graph.  prm: as for sample_sort_pairs (NULL = tuned). */
int ss_strings_workspace_size(size_t n, uint32_t width, const ss_params *prm, size_t *bytes_out);
int sample_sort_strings(const void *recs, void *recs_out, int64_t *perm_out, size_t n, uint32_t width,
                        const ss_params *prm, void *ws, size_t ws_bytes, void *stream);

/* Workspace bytes for segmented_sort: `total` keys in `num_segments`
 * segments, none longer than `max_seg_len` (0 = unknown, taken as total). */
int ss_segmented_workspace_size(size_t total, size_t num_segments, size_t max_seg_len, int key_type,
                                int val_type, const ss_params *prm, size_t *bytes_out);

/* Sort every segment [offsets[g], offsets[g+1]) independently (stable), for
 * g < num_segments, in one fixed sequence of kernel launches whatever the
 * segment sizes (so the call can be captured into a HIP graph and replayed).
 * d_offsets: DEVICE int64[num_segments+1], non-decreasing, offsets[0] may be
 * > 0; `total` must equal offsets[num_segments] and `max_seg_len` bound
 * every segment length (both host values).  Empty segments are allowed.  For
 * the IOTA payload types the payload is the index within the segment.
 * prm may be NULL: then each segment takes p and s of its size class from
 * the tuning table (ss_set_tuning); otherwise prm->s, prm->seed and
 * prm->tile apply to every split, and prm->p caps the buckets per segment.
 * Segments below one split level are sorted in three classes: up to 64
 * keys by one wave each, up to 2048 by a work-group with a small LDS
 * footprint, the rest by a work-group with the full LDS. */
int segmented_sort(const void *keys_in, const void *vals_in, void *keys_out, void *vals_out,
                   const int64_t *d_offsets, size_t num_segments, size_t total, size_t max_seg_len,
                   int key_type, int val_type, const ss_params *prm, void *ws, size_t ws_bytes,
                   void *stream);

/* Parameters that a call with prm == NULL uses (tuned defaults).  The paper
 * fixes p for the machine after calibration and ties the sample size to n
 * (Section 2.1, Section 3); here each size class of the length (class c:
 * lengths in (2^(c-1), 2^c]) has its own (p, s, tile), per form (single
 * array or segmented), key width and payload width as sorted (a 64-bit
 * index payload counts as 4 bytes).  A single sort of n keys uses the
 * class of n; segmented_sort uses each segment's class for its buckets and
 * oversampling (tile: the class of max_seg_len).  Sampling is random
 * (Alg. 2), seed 0x5EED.  The library holds a built-in table measured on an
 * MI355X; paper_1608_08648_amd.tune measures a new one and installs it. */
typedef struct ss_tune_entry {
    uint32_t form;        /* 0 = sample_sort_keys / sample_sort_pairs, 1 = segmented_sort */
    uint32_t key_bytes;   /* 4 or 8 */
    uint32_t val_bytes;   /* 0, 4 or 8 */
    uint32_t size_class;  /* 0..32 */
    uint32_t p;           /* power of two in [2, SS_P_MAX]; segmented only: 0 = sized from the length */
    uint32_t s;           /* 1..4096 */
    uint32_t tile;        /* keys per work-group in the split passes, 0 = chosen per p */
} ss_tune_entry;

/* Replace the table prm == NULL uses: the built-in table overwritten by
 * `count` entries (count = 0 restores the built-in table).  Host only; an
 * invalid entry leaves the table unchanged (SS_EINVAL).  Calls already
 * enqueued are not affected; calls racing with this one see either table. */
int ss_set_tuning(const ss_tune_entry *entries, size_t count);

/* The parameters a prm == NULL call of form `form` (0 single, 1 segmented)
 * on n keys (segmented: a segment of n keys) of these types would use.
 * Host only.  For the segmented form p = 256 stands for "sized from the
 * length, at most 256". */
int ss_get_tuning(int form, int key_type, int val_type, size_t n, ss_params *out);

/* Backward of a row-wise sort y[r, j] = x[r, perm[r, j]]: the gradient goes
 * back through the permutation, grad_x[r, perm[r, j]] = grad_y[r, j].  Each
 * row of perm must be a permutation of 0..row_len-1 (then every grad_x
 * element is written exactly once); an index outside [0, row_len) is not
 * written and is reported by ss_grad_status.  elem_bytes = 2, 4 or 8.
 * grad_y, grad_x: device [rows, row_len]; perm: device int64 [rows,
 * row_len]; grad_y and perm 16-byte aligned; rows, row_len < 2^31. */
int ss_scatter_grad(const void *grad_y, const int64_t *perm, void *grad_x, size_t rows, size_t row_len,
                    int elem_bytes, void *stream);

/* Wait for `stream`, then report whether any ss_scatter_grad call since the
 * last ss_grad_status met an index outside its row (SS_EDEVICE, and the
 * flag is cleared) or not (SS_OK).  The flag is one per process and
 * device, shared by all calls. */
int ss_grad_status(void *stream);

/* Wait for `stream`, then read the device status word of the last call that
 * used `ws`: SS_OK, or SS_EDEVICE if the device reported a condition (the
 * message names it). */
int ss_status(const void *ws, void *stream);

/* Split levels.  A bucket that the in-work-group bucket sorts cannot take
 * (Lemma 1 bounds its size only in expectation-scaled terms, and a skewed
 * input can exceed any fixed capacity) is sample-sorted again, by the next
 * level, with its own sample and splitters; level 0 splits the whole input
 * (or, for segmented_sort, the segments too long for one work-group). */
#define SS_MAX_LEVELS 6

typedef struct {
  uint32_t segments;     /* segments the level split */
  uint32_t buckets;      /* buckets they were split into */
  uint64_t keys;         /* keys in those segments */
  uint64_t bucket_keys;  /* of those, keys that the level's bucket kernel sorted in place;
                            the rest went to the next level or to the larger-bucket sorts */
} ss_level_info;

/* Wait for `stream`, then fill *info with the counts of split level `level`
 * (0 <= level < SS_MAX_LEVELS) of the last call that used `ws` (a
 * diagnostic: how deep the recursion went and how much data each level
 * moved).  Levels the call did not reach read as zero.  SS_EINVAL for a
 * NULL pointer or a level out of range. */
int ss_level_stats(const void *ws, int level, ss_level_info *info, void *stream);

/* Per-kernel timing, for benchmarks.  While enabled (on != 0), every kernel
 * the library launches is bracketed by two HIP events recorded on the
 * caller's stream (from a pool of `max_launches` event pairs created here;
 * this call may allocate host/driver resources and must not be made during
 * graph capture).  ss_profile_collect() waits for the recorded events and
 * adds their durations to per-kernel totals; ss_profile_report(i, ...)
 * returns the name, total milliseconds and launch count of kernel kind i
 * (SS_EINVAL past the last kind).  ss_profile_enable(0) frees the pool and
 * clears the totals.  ss_profile_kinds(mask) limits the bracketing to the
 * kinds whose bit (1 << i) is set (every kind after ss_profile_enable), so
 * that a timed run records events only around the kernels it measures. */
int ss_profile_enable(int on, int max_launches);
int ss_profile_kinds(unsigned kind_mask);
int ss_profile_collect(void);
int ss_profile_report(int kind, const char **name, double *total_ms, uint64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* SAMPLESORT_H */
