/*
 * CPU oracle for the oversampling sample sort of Gerbessiotis,
 * "Using parallelism techniques to improve sequential and multi-core
 * sorting performance" (arXiv 1608.08648).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file: only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header, table or constant with
 * the HIP library; the two meet only through the seeded input generators.
 *
 * Plain, slow, single-threaded and written to be checked against the paper
 * by eye:
 *   - orc_stable_sort: the definition of the result.  Section 1 defines a
 *     stable sort as one in which equal keys keep their relative input
 *     order, so the output is the input permuted by the unique pi with
 *     (key[pi(0)], pi(0)) < (key[pi(1)], pi(1)) < ...  A top-down merge
 *     sort that takes the left run on ties computes exactly that.
 *   - orc_stages: the method's steps in the paper's order (sample,
 *     sort the sample, pick splitters, split the keys, sort each part,
 *     concatenate), in the traditional sample-first organisation that
 *     Section 1 and the discussion after Claim 1 describe, with the
 *     duplicate-key tags of Section 2.2.
 *
 * Keys are compared through an order-preserving map to unsigned 64-bit
 * integers (ord): unsigned keys as they are, signed keys with the sign bit
 * flipped, IEEE floats by the totalOrder bit trick (negative values have
 * all bits flipped, non-negative ones only the sign bit).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ORC_PLANT selects a deliberate mistake for the tests that show the pins
 * catch it (0 = the correct oracle; see tests/test_oracle_plants.py). */
#ifndef ORC_PLANT
#define ORC_PLANT 0
#endif

enum { ORC_U32 = 0, ORC_I32 = 1, ORC_F32 = 2, ORC_U64 = 3, ORC_I64 = 4, ORC_F64 = 5 };
enum { ORC_RANDOM = 0, ORC_REGULAR = 1 };

/* ------------------------------------------------------------------ keys */

static uint64_t ord32(uint32_t u, int kt)
{
    if (kt == ORC_I32) return (uint64_t)(ORC_PLANT == 6 ? u : (u ^ 0x80000000u));
    if (kt == ORC_F32) return (uint64_t)((u & 0x80000000u) ? ~u : (u ^ 0x80000000u));
    return (uint64_t)u;
}

static uint64_t ord64(uint64_t u, int kt)
{
    if (kt == ORC_I64) return u ^ 0x8000000000000000ull;
    if (kt == ORC_F64) return (u & 0x8000000000000000ull) ? ~u : (u ^ 0x8000000000000000ull);
    return u;
}

static int key_bytes(int kt) { return (kt <= ORC_F32) ? 4 : 8; }

/* ord of key i of an array of key type kt */
uint64_t orc_ord(const void *keys, uint64_t i, int kt)
{
    if (key_bytes(kt) == 4) {
        uint32_t u;
        memcpy(&u, (const char *)keys + 4 * i, 4);
        return ord32(u, kt);
    } else {
        uint64_t u;
        memcpy(&u, (const char *)keys + 8 * i, 8);
        return ord64(u, kt);
    }
}

/* A record: the key's ord plus the tag that breaks ties (Section 2.2 tags
 * each sampled key with where it sits in the input; here the tag is the
 * input index). */
typedef struct { uint64_t ord; uint64_t tag; } rec_t;

static int rec_less(const rec_t *a, const rec_t *b)
{
    if (a->ord != b->ord) return a->ord < b->ord;
    return (ORC_PLANT == 5) ? 0 : a->tag < b->tag;
}

/* --------------------------------------------------- stable merge sort */

/* Sort a[0..n) by ord only; on equal ord the left run's record goes first,
 * so records with equal keys keep their input order (stability). */
static void merge_sort_by_ord(rec_t *a, rec_t *tmp, uint64_t n)
{
    if (n < 2) return;
    uint64_t h = n / 2;
    merge_sort_by_ord(a, tmp, h);
    merge_sort_by_ord(a + h, tmp, n - h);
    uint64_t i = 0, j = h, k = 0;
    while (i < h && j < n) {
        if (ORC_PLANT == 1 ? a[j].ord <= a[i].ord : a[j].ord < a[i].ord) tmp[k++] = a[j++];
        else tmp[k++] = a[i++];
    }
    while (i < h) tmp[k++] = a[i++];
    while (j < n) tmp[k++] = a[j++];
    memcpy(a, tmp, n * sizeof(rec_t));
}

/* Sort a[0..n) by (ord, tag): used for the sample, whose records are not in
 * tag order when drawn. */
static void merge_sort_by_rec(rec_t *a, rec_t *tmp, uint64_t n)
{
    if (n < 2) return;
    uint64_t h = n / 2;
    merge_sort_by_rec(a, tmp, h);
    merge_sort_by_rec(a + h, tmp, n - h);
    uint64_t i = 0, j = h, k = 0;
    while (i < h && j < n) {
        if (rec_less(&a[j], &a[i])) tmp[k++] = a[j++];
        else tmp[k++] = a[i++];
    }
    while (i < h) tmp[k++] = a[i++];
    while (j < n) tmp[k++] = a[j++];
    memcpy(a, tmp, n * sizeof(rec_t));
}

/* The definition: perm[r] = input index of the r-th record of the stable
 * ascending order.  Returns 0, or -1 if memory runs out. */
int orc_stable_sort(const void *keys, uint64_t n, int kt, uint64_t *perm)
{
    rec_t *a = (rec_t *)malloc((n ? n : 1) * sizeof(rec_t));
    rec_t *t = (rec_t *)malloc((n ? n : 1) * sizeof(rec_t));
    if (!a || !t) { free(a); free(t); return -1; }
    for (uint64_t i = 0; i < n; i++) { a[i].ord = orc_ord(keys, i, kt); a[i].tag = i; }
    merge_sort_by_ord(a, t, n);
    for (uint64_t i = 0; i < n; i++) perm[i] = a[i].tag;
    free(a);
    free(t);
    return 0;
}

/* Segmented form: each segment [off[g], off[g+1]) is sorted on its own;
 * perm holds in-segment indices. */
int orc_segmented_sort(const void *keys, const int64_t *off, uint64_t nseg, int kt, uint64_t *perm)
{
    int kb = key_bytes(kt);
    for (uint64_t g = 0; g < nseg; g++) {
        uint64_t b = (uint64_t)off[g], e = (uint64_t)off[g + 1];
        if (e < b) return -2;
        if (orc_stable_sort((const char *)keys + kb * b, e - b, kt, perm + b) != 0) return -1;
    }
    return 0;
}

/* ------------------------------------------------------------ SplitMix64 */

/* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014; the variant with the
 * 30/27/31 shift finaliser used by java.util.SplittableRandom): the state
 * advances by the golden-ratio increment and each output is the finaliser
 * applied to the new state. */
static uint64_t sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static const uint64_t SM64_GAMMA = 0x9E3779B97F4A7C15ull;

/* The first cnt outputs of a SplitMix64 generator whose state is seed. */
void orc_splitmix64(uint64_t seed, uint64_t cnt, uint64_t *out)
{
    uint64_t st = seed;
    for (uint64_t j = 0; j < cnt; j++) {
        st += SM64_GAMMA;
        out[j] = sm64_mix(st);
    }
}

/* floor(r * n / 2^64): maps a 64-bit uniform word to [0, n). */
static uint64_t scale_to(uint64_t r, uint64_t n)
{
    return (uint64_t)(((unsigned __int128)r * (unsigned __int128)n) >> 64);
}

/* --------------------------------------------------------- parameters */

/* Effective bucket count: the largest power of two <= p that keeps the
 * preconditions the paper states: p <= n (Theorem 1); for random
 * oversampling p*s < n/2 (Claim 1); for regular oversampling a sample of
 * s*p^2 that is small against n (Theorem 1 asks p^2 w^2 = o(n); read
 * here as 4*s*p^2 <= n).  Returns 1 when no p >= 2 qualifies, in which
 * case the keys are sorted directly. */
uint32_t orc_p_eff(uint64_t n, uint32_t p, uint32_t s, int mode)
{
    uint64_t q = 1;
    while (q * 2 <= p) q *= 2;
    for (; q >= 2; q /= 2) {
        if (q > n) continue;
        if (mode == ORC_RANDOM) {
            if (2 * q * (uint64_t)s < n) return (uint32_t)q;
        } else {
            if (4 * (uint64_t)s * q * q <= n) return (uint32_t)q;
        }
    }
    return 1;
}

/* ------------------------------------------------------- staged method */

/* Number of sample records the method draws. */
uint64_t orc_sample_count(uint32_t p, uint32_t s, int mode)
{
    if (mode == ORC_RANDOM) return (uint64_t)p * s - 1;         /* Alg. 2, step 2 */
    return (uint64_t)s * p * p;                                  /* Alg. 1, step 2: r*p per block */
}

/* Draw the sample (Alg. 2 step 2 or Alg. 1 steps 1-2) into smp[0..m).
 *  RANDOM:  sample j is the record at position pos_j, where pos_j scales the
 *           (j+1)-th SplitMix64 output of `seed` to [0, n) (with
 *           replacement).
 *  REGULAR: block k = [floor(k n/p), floor((k+1) n/p)), sorted by (ord, tag)
 *           (Alg. 1 step 1); with S = s*p and x = ceil(ceil(n/p)/S) (the
 *           segment length of the padded block in the proof of Lemma 1),
 *           sample j of block k is the block's record of rank
 *           min((j+1)*x, |block|) - 1: S-1 evenly spaced keys and the block
 *           maximum.  Padding is never materialised: a padded rank maps to
 *           the block's largest record. */
static int draw_sample(const void *keys, uint64_t n, int kt, uint32_t p, uint32_t s, int mode,
                       uint64_t seed, rec_t *smp)
{
    if (mode == ORC_RANDOM) {
        uint64_t m = (uint64_t)p * s - 1;
        uint64_t *r = (uint64_t *)malloc((m ? m : 1) * sizeof(uint64_t));
        if (!r) return -1;
        orc_splitmix64(seed, m, r);
        for (uint64_t j = 0; j < m; j++) {
            uint64_t pos = scale_to(r[j], n);
            smp[j].ord = orc_ord(keys, pos, kt);
            smp[j].tag = pos;
        }
        free(r);
        return 0;
    }
    uint64_t S = (uint64_t)s * p;
    uint64_t blk_max = (n + p - 1) / p;               /* ceil(n/p) */
    uint64_t x = (ORC_PLANT == 4) ? blk_max / S : (blk_max + S - 1) / S;  /* ceil(ceil(n/p)/S) */
    if (x == 0) x = 1;
    rec_t *blk = (rec_t *)malloc((blk_max ? blk_max : 1) * sizeof(rec_t));
    rec_t *tmp = (rec_t *)malloc((blk_max ? blk_max : 1) * sizeof(rec_t));
    if (!blk || !tmp) { free(blk); free(tmp); return -1; }
    for (uint64_t k = 0; k < p; k++) {
        uint64_t b = (k * n) / p, e = ((k + 1) * n) / p, mk = e - b;
        for (uint64_t i = 0; i < mk; i++) { blk[i].ord = orc_ord(keys, b + i, kt); blk[i].tag = b + i; }
        merge_sort_by_rec(blk, tmp, mk);
        for (uint64_t j = 0; j < S; j++) {
            uint64_t rank = (j + 1) * x;
            if (rank > mk) rank = mk;
            smp[k * S + j] = blk[rank - 1];
        }
    }
    free(blk);
    free(tmp);
    return 0;
}

/* bucket(e) = #{ i : spl_i < e } over the p-1 sorted splitters, comparing
 * records by key and then by tag (Section 2.2: split by key first, tags
 * only when keys are equal).  A splitter closes its own bucket. */
static uint64_t bucket_of(const rec_t *spl, uint64_t nspl, const rec_t *e)
{
    uint64_t lo = 0, hi = nspl;             /* count = first index with !(spl < e) */
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (ORC_PLANT == 3 ? !rec_less(e, &spl[mid]) : rec_less(&spl[mid], e)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

/*
 * Run the method step by step for one top-level pass and finish by sorting
 * each bucket.  Outputs (all optional, may be NULL):
 *   smp_ord/smp_tag[m]  the sorted sample (m = orc_sample_count)
 *   spl_ord/spl_tag[p-1] the splitters
 *   counts[p]           keys per bucket
 *   perm[n]             the concatenation of the sorted buckets, as input
 *                       indices
 * p must already be the effective bucket count (>= 2, a power of two).
 */
int orc_stages(const void *keys, uint64_t n, int kt, uint32_t p, uint32_t s, int mode, uint64_t seed,
               uint64_t *smp_ord, uint64_t *smp_tag, uint64_t *spl_ord, uint64_t *spl_tag,
               uint64_t *counts, uint64_t *perm)
{
    if (p < 2 || (p & (p - 1)) || s < 1 || n < 1) return -2;
    uint64_t m = orc_sample_count(p, s, mode);
    uint64_t stride = (mode == ORC_RANDOM) ? (uint64_t)s : (uint64_t)s * p;
    int rc = -1;
    rec_t *smp = (rec_t *)malloc(m * sizeof(rec_t));
    rec_t *tmp = (rec_t *)malloc((m > n ? m : n) * sizeof(rec_t));
    rec_t *spl = (rec_t *)malloc((p - 1) * sizeof(rec_t));
    uint64_t *cnt = (uint64_t *)calloc(p, sizeof(uint64_t));
    uint64_t *start = (uint64_t *)malloc((p + 1) * sizeof(uint64_t));
    uint64_t *bkt = (uint64_t *)malloc(n * sizeof(uint64_t));
    rec_t *part = (rec_t *)malloc(n * sizeof(rec_t));
    if (!smp || !tmp || !spl || !cnt || !start || !bkt || !part) goto out;

    /* step 2: draw and sort the sample by (key, tag) */
    if (draw_sample(keys, n, kt, p, s, mode, seed, smp) != 0) goto out;
    merge_sort_by_rec(smp, tmp, m);
    if (smp_ord) for (uint64_t j = 0; j < m; j++) smp_ord[j] = smp[j].ord;
    if (smp_tag) for (uint64_t j = 0; j < m; j++) smp_tag[j] = smp[j].tag;

    /* step 3: splitter i (1-based) is the (i*stride)-th smallest sample */
    for (uint64_t i = 1; i < p; i++) spl[i - 1] = smp[i * stride - (ORC_PLANT == 2 ? 0 : 1)];
    if (spl_ord) for (uint64_t i = 0; i + 1 < p; i++) spl_ord[i] = spl[i].ord;
    if (spl_tag) for (uint64_t i = 0; i + 1 < p; i++) spl_tag[i] = spl[i].tag;

    /* step 4: split every key around the splitters */
    for (uint64_t i = 0; i < n; i++) {
        rec_t e;
        e.ord = orc_ord(keys, i, kt);
        e.tag = i;
        bkt[i] = bucket_of(spl, p - 1, &e);
        cnt[bkt[i]]++;
    }
    if (counts) for (uint64_t b = 0; b < p; b++) counts[b] = cnt[b];

    /* bucket b occupies [start[b], start[b+1]) of the concatenation; place
     * keys in input order (a stable scatter) */
    start[0] = 0;
    for (uint64_t b = 0; b < p; b++) start[b + 1] = start[b] + cnt[b];
    for (uint64_t b = 0; b < p; b++) cnt[b] = 0;
    for (uint64_t i = 0; i < n; i++) {
        uint64_t b = bkt[i];
        part[start[b] + cnt[b]].ord = orc_ord(keys, i, kt);
        part[start[b] + cnt[b]].tag = i;
        cnt[b]++;
    }

    /* step 5 (sample-first form): sort each bucket stably; the buckets
     * concatenate into the output */
    for (uint64_t b = 0; b < p; b++)
        merge_sort_by_ord(part + start[b], tmp, start[b + 1] - start[b]);
    if (perm) for (uint64_t i = 0; i < n; i++) perm[i] = part[i].tag;
    rc = 0;
out:
    free(smp); free(tmp); free(spl); free(cnt); free(start); free(bkt); free(part);
    return rc;
}

/* ord of every key (for the tests of the key order) */
void orc_ord_array(const void *keys, uint64_t n, int kt, uint64_t *out)
{
    for (uint64_t i = 0; i < n; i++) out[i] = orc_ord(keys, i, kt);
}

/* ----------------------------------------------------------- Lemma 1 */

/* Bucket-size bounds of Lemma 1 (Section 2.1) for regular oversampling
 * with factor r (the API's s) and p buckets.  The proof pads every block to
 * ceil(n/p) keys and cuts it into S = r*p segments of
 * x = ceil(ceil(n/p)/S) keys; a splitter has at least i*S*x keys below it
 * and at least (p*S - i*S - p + 1)*x above it, so two neighbouring
 * splitters enclose at most S*x + p*x - x keys.
 *   out_u[0] = (S + p) * x       the bound with the "- x" dropped
 *   out_u[1] = (S + p - 1) * x   the difference bound b_{i+1} - b_i
 *   out_d[0] = (1 + 1/r) * n/p + r*p, the lemma's closing expression. */
void orc_lemma1(uint64_t n, uint32_t p, uint32_t r, uint64_t *out_u, double *out_d)
{
    uint64_t S = (uint64_t)r * p;
    uint64_t blk = (n + p - 1) / p;                                   /* ceil(n/p) */
    uint64_t x = (ORC_PLANT == 7) ? blk / S : (blk + S - 1) / S;      /* ceil(blk/S) */
    out_u[0] = (S + p) * x;
    out_u[1] = (S + p - 1) * x;
    out_d[0] = (1.0 + 1.0 / (double)r) * (double)n / (double)p + (double)r * (double)p;
}

/* ------------------------------------------------------ byte-string keys */

/* The paper's measured keys are strings of 32 bytes compared as memcmp
 * does (Section 3): byte by byte as unsigned values, the first differing
 * byte deciding.  orc_stable_sort_bytes is the definition of the stable
 * result for n records of `width` bytes: the unique permutation with
 * (record, index) strictly increasing, by a top-down merge sort of the
 * indices that takes the left run on ties. */
static const uint8_t *g_recs;
static uint32_t g_width;

static int rec_bytes_less(uint64_t a, uint64_t b)
{
    const uint32_t w = (ORC_PLANT == 8 && g_width > 8) ? 8 : g_width;
    int c = memcmp(g_recs + a * g_width, g_recs + b * g_width, w);
    return c < 0;
}

static void merge_sort_idx(uint64_t *a, uint64_t *tmp, uint64_t n)
{
    if (n < 2) return;
    uint64_t h = n / 2;
    merge_sort_idx(a, tmp, h);
    merge_sort_idx(a + h, tmp, n - h);
    uint64_t i = 0, j = h, k = 0;
    while (i < h && j < n) {
        /* right before left only if strictly smaller: ties keep input order */
        if (rec_bytes_less(a[j], a[i])) tmp[k++] = a[j++];
        else tmp[k++] = a[i++];
    }
    while (i < h) tmp[k++] = a[i++];
    while (j < n) tmp[k++] = a[j++];
    memcpy(a, tmp, n * sizeof(uint64_t));
}

int orc_stable_sort_bytes(const uint8_t *recs, uint64_t n, uint32_t width, uint64_t *perm)
{
    uint64_t *tmp = (uint64_t *)malloc((n ? n : 1) * sizeof(uint64_t));
    if (!tmp) return -1;
    for (uint64_t i = 0; i < n; i++) perm[i] = i;
    g_recs = recs;
    g_width = width;
    merge_sort_idx(perm, tmp, n);
    free(tmp);
    return 0;
}
