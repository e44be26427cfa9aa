/*
 * Host multi-core comparator: the paper's McRan (random oversampling,
 * sort-first organisation, step 1 spread over threads), on the host CPU.
 *
 * A CPU reference point for the GPU sort, measured on the same machine: it
 * is never called by the GPU sort and shares no code with it.  It follows
 * Alg. 2 with the multi-core adaptation of the section on multi-core
 * variants:
 *   1. split the n keys into p blocks of about n/p keys and sort each block
 *      with SomeSort (here the C library's qsort); the p sorts are spread
 *      over t threads (t <= p);
 *   2. draw a sample of p*s - 1 keys uniformly at random (with replacement)
 *      and sort it with SomeSort;
 *   3. take the (i*s)-th smallest sample keys, 1 <= i <= p-1, as splitters;
 *   4. split every sorted block around the splitters by binary search
 *      (run j of block k holds its keys in (splitter j, splitter j+1]);
 *   5. merge the p runs of every bucket j (a p-way merge through a binary
 *      heap) into its place in the output; the buckets concatenate to the
 *      sorted output.  As in the paper's measurements step 5 runs on one
 *      thread unless merge_threads > 1 spreads the buckets over threads.
 * Keys are 32-bit signed integers (the GPU benchmark's key type); equal
 * keys are interchangeable, so no tags are needed for a keys-only result.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

typedef struct {
    int32_t *a;
    const uint64_t *bnd;      /* p + 1 block bounds */
    uint32_t p, t, id;
} blk_job;

static int cmp_i32(const void *x, const void *y)
{
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

static void *sort_blocks(void *arg)
{
    blk_job *j = (blk_job *)arg;
    for (uint32_t k = j->id; k < j->p; k += j->t)
        qsort(j->a + j->bnd[k], j->bnd[k + 1] - j->bnd[k], sizeof(int32_t), cmp_i32);
    return NULL;
}

/* SplitMix64 (Steele, Lea, Flood): the sample positions */
static uint64_t mix64(uint64_t *st)
{
    uint64_t z = (*st += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* first index in a[0, len) whose key is > v */
static uint64_t upper(const int32_t *a, uint64_t len, int32_t v)
{
    uint64_t lo = 0, hi = len;
    while (lo < hi) {
        uint64_t m = lo + (hi - lo) / 2;
        if (a[m] <= v) lo = m + 1;
        else hi = m;
    }
    return lo;
}

typedef struct {
    const int32_t *a;         /* sorted blocks */
    const uint64_t *bnd;      /* block bounds */
    const uint64_t *cut;      /* cut[k * (p + 1) + j]: start of run j in block k (absolute) */
    const uint64_t *ystart;   /* output start of bucket j */
    int32_t *y;
    uint32_t p, t, id;
} merge_job;

/* p-way merge of the runs of bucket j through a binary min-heap of
 * (key, block) heads. */
static void merge_bucket(const merge_job *m, uint32_t j, uint64_t *pos, uint32_t *heap)
{
    const uint32_t p = m->p;
    uint32_t hn = 0;
    for (uint32_t k = 0; k < p; k++) {
        pos[k] = m->cut[(uint64_t)k * (p + 1) + j];
        if (pos[k] < m->cut[(uint64_t)k * (p + 1) + j + 1]) {
            uint32_t c = hn++;
            heap[c] = k;
            while (c) {                                   /* sift up */
                uint32_t par = (c - 1) / 2;
                if (m->a[pos[heap[par]]] <= m->a[pos[heap[c]]]) break;
                uint32_t tmp = heap[par]; heap[par] = heap[c]; heap[c] = tmp;
                c = par;
            }
        }
    }
    uint64_t o = m->ystart[j];
    while (hn) {
        uint32_t k = heap[0];
        m->y[o++] = m->a[pos[k]++];
        if (pos[k] == m->cut[(uint64_t)k * (p + 1) + j + 1]) heap[0] = heap[--hn];
        uint32_t c = 0;                                   /* sift down */
        for (;;) {
            uint32_t l = 2 * c + 1, r = l + 1, b = c;
            if (l < hn && m->a[pos[heap[l]]] < m->a[pos[heap[b]]]) b = l;
            if (r < hn && m->a[pos[heap[r]]] < m->a[pos[heap[b]]]) b = r;
            if (b == c) break;
            uint32_t tmp = heap[b]; heap[b] = heap[c]; heap[c] = tmp;
            c = b;
        }
    }
}

static void *merge_buckets(void *arg)
{
    merge_job *m = (merge_job *)arg;
    uint64_t *pos = (uint64_t *)malloc(sizeof(uint64_t) * m->p);
    uint32_t *heap = (uint32_t *)malloc(sizeof(uint32_t) * m->p);
    if (pos && heap)
        for (uint32_t j = m->id; j < m->p; j += m->t) merge_bucket(m, j, pos, heap);
    free(pos);
    free(heap);
    return NULL;
}

static double now_s(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return ts.tv_sec + 1e-9 * ts.tv_nsec;
}

/*
 * Sort x[0, n) into y[0, n) (x is sorted block-wise in place).  p >= 1
 * buckets (p <= n), s >= 1, threads >= 1 sort threads (at most p),
 * merge_threads >= 1.  times[0..4] (optional) receive the seconds spent in
 * steps 1, 2 (with 3), 4 and 5.  Returns 0, or -1 on bad arguments or
 * failed allocation.
 */
int mcran_sort_i32(int32_t *x, int32_t *y, uint64_t n, uint32_t p, uint32_t s, uint64_t seed, uint32_t threads,
                   uint32_t merge_threads, double *times)
{
    if (!x || !y || p < 1 || s < 1 || threads < 1 || merge_threads < 1) return -1;
    if (n == 0) return 0;
    if (p > n) p = (uint32_t)n;
    if (threads > p) threads = p;
    if (merge_threads > p) merge_threads = p;
    double t0 = now_s();
    uint64_t *bnd = (uint64_t *)malloc(sizeof(uint64_t) * (p + 1));
    uint64_t *cut = (uint64_t *)malloc(sizeof(uint64_t) * (uint64_t)p * (p + 1));
    uint64_t *ystart = (uint64_t *)malloc(sizeof(uint64_t) * (p + 1));
    const uint64_t m = (uint64_t)p * s - 1;
    int32_t *smp = (int32_t *)malloc(sizeof(int32_t) * (m ? m : 1));
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (threads > merge_threads ? threads : merge_threads));
    blk_job *bj = (blk_job *)malloc(sizeof(blk_job) * threads);
    merge_job *mj = (merge_job *)malloc(sizeof(merge_job) * merge_threads);
    int rc = -1;
    if (!bnd || !cut || !ystart || !smp || !th || !bj || !mj) goto out;
    /* step 1: p blocks of about n/p keys, sorted by t threads */
    for (uint32_t k = 0; k <= p; k++) bnd[k] = (uint64_t)k * n / p;
    for (uint32_t i = 0; i < threads; i++) {
        bj[i] = (blk_job){x, bnd, p, threads, i};
        if (i) pthread_create(&th[i], NULL, sort_blocks, &bj[i]);
    }
    sort_blocks(&bj[0]);
    for (uint32_t i = 1; i < threads; i++) pthread_join(th[i], NULL);
    double t1 = now_s();
    /* steps 2-3: random sample, sorted; splitters are its (i*s)-th smallest */
    uint64_t st = seed;
    for (uint64_t i = 0; i < m; i++) {
        uint64_t r = mix64(&st);
        uint64_t pos = (uint64_t)(((unsigned __int128)r * n) >> 64);
        smp[i] = x[pos];
    }
    qsort(smp, m, sizeof(int32_t), cmp_i32);
    double t2 = now_s();
    /* step 4: cut every sorted block at the splitters; bucket j takes keys
     * in (splitter j, splitter j+1] (splitter i = smp[i*s - 1]) */
    for (uint32_t j = 0; j <= p; j++) ystart[j] = 0;
    for (uint32_t k = 0; k < p; k++) {
        const int32_t *blk = x + bnd[k];
        const uint64_t len = bnd[k + 1] - bnd[k];
        uint64_t *c = cut + (uint64_t)k * (p + 1);
        c[0] = bnd[k];
        for (uint32_t j = 1; j < p; j++) c[j] = bnd[k] + upper(blk, len, smp[(uint64_t)j * s - 1]);
        c[p] = bnd[k + 1];
        for (uint32_t j = 0; j < p; j++) ystart[j + 1] += c[j + 1] - c[j];
    }
    for (uint32_t j = 0; j < p; j++) ystart[j + 1] += ystart[j];
    double t3 = now_s();
    /* step 5: merge each bucket's p runs into its place in y */
    for (uint32_t i = 0; i < merge_threads; i++) {
        mj[i] = (merge_job){x, bnd, cut, ystart, y, p, merge_threads, i};
        if (i) pthread_create(&th[i], NULL, merge_buckets, &mj[i]);
    }
    merge_buckets(&mj[0]);
    for (uint32_t i = 1; i < merge_threads; i++) pthread_join(th[i], NULL);
    double t4 = now_s();
    if (times) {
        times[0] = t1 - t0;
        times[1] = t2 - t1;
        times[2] = t3 - t2;
        times[3] = t4 - t3;
        times[4] = t4 - t0;
    }
    rc = 0;
out:
    free(bnd); free(cut); free(ystart); free(smp); free(th); free(bj); free(mj);
    return rc;
}
