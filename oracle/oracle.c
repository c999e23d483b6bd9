/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU implementation of what the paper's
 * "scatter / sort / merge" method computes (El-Nashar, IJDPS 2(3) 2011,
 * Section 3.2 and Figures 1-3).  It exists to check the GPU library and must
 * never be used by it: only the tests, the smoke check and the benchmark's
 * CPU-baseline leg load this file's shared object.  It shares no code, header,
 * table or helper with the HIP path.
 *
 * What is computed (the plain definition the method reaches exactly):
 *   given keys k[0..n) (and optional 32-bit values v[0..n)), the output is the
 *   unique permutation pi of [0, n) with k[pi(0)] <= k[pi(1)] <= ... in the key
 *   type's natural order (signed for int32, unsigned for uint32 / uint64) and,
 *   for equal keys, pi(i) < pi(i+1): the stable ascending sort.  Values travel
 *   with their keys.
 *
 * How it is computed: the top-down merge sort of Figure 3, with the garbled
 * outline repaired (one index name for the range start, floor midpoint, an
 * explicit empty-range base case, one scratch buffer allocated once instead of
 * a fresh pair of sub-lists at every level), and a merge that takes the left
 * run's item whenever the two are equal (the tie rule that makes the sort
 * stable; the paper never shows the merge body).
 *
 * Everything is done on 64-bit "raw bit" records so one code path serves all
 * three key types; the comparison interprets the raw bits per key type.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

/* Key type codes (0 = int32, 1 = uint32, 2 = uint64). */
enum { ORACLE_I32 = 0, ORACLE_U32 = 1, ORACLE_U64 = 2 };

/* One list item: the key's raw bits (zero-extended) and its value. */
struct item {
    uint64_t key;
    uint32_t val;
};

/* a <= b in the natural order of key type kt.  Section 3.2 leaves the order
 * implicit; Figure 2 swaps when the left item is greater, i.e. ascending. */
static int key_le(int kt, uint64_t a, uint64_t b)
{
    if (kt == ORACLE_I32)
        return (int32_t)(uint32_t)a <= (int32_t)(uint32_t)b;
    return a <= b; /* uint32 (zero-extended) and uint64 */
}

static int key_lt(int kt, uint64_t a, uint64_t b) { return !key_le(kt, b, a); }

static int valid_kt(int kt) { return kt == ORACLE_I32 || kt == ORACLE_U32 || kt == ORACLE_U64; }

static size_t key_bytes(int kt) { return kt == ORACLE_U64 ? 8 : 4; }

static uint64_t load_key(int kt, const void *keys, uint64_t i)
{
    if (kt == ORACLE_U64)
        return ((const uint64_t *)keys)[i];
    return ((const uint32_t *)keys)[i];
}

static void store_key(int kt, void *keys, uint64_t i, uint64_t bits)
{
    if (kt == ORACLE_U64)
        ((uint64_t *)keys)[i] = bits;
    else
        ((uint32_t *)keys)[i] = (uint32_t)bits;
}

/* Read n items; values default to 0 when the caller passes none. */
static struct item *read_items(int kt, const void *keys, const uint32_t *vals, uint64_t n)
{
    struct item *a = (struct item *)malloc((n ? n : 1) * sizeof(struct item));
    if (!a)
        return NULL;
    for (uint64_t i = 0; i < n; i++) {
        a[i].key = load_key(kt, keys, i);
        a[i].val = vals ? vals[i] : 0u;
    }
    return a;
}

static void write_items(int kt, const struct item *a, uint64_t n, void *keys, uint32_t *vals)
{
    for (uint64_t i = 0; i < n; i++) {
        store_key(kt, keys, i, a[i].key);
        if (vals)
            vals[i] = a[i].val;
    }
}

/* ------------------------------------------------------------------------ */
/* Figure 3: merge two adjacent sorted runs a[first..mid] and a[mid+1..last]
 * (inclusive bounds).  lcount and ucount are the two run lengths exactly as
 * Figure 3 defines them.  While both runs have items, the left run's item is
 * taken when it is <= the right run's (left first on ties); then the tail of
 * whichever run remains is copied. */
static void merge_adjacent(int kt, struct item *a, struct item *scratch,
                           uint64_t first, uint64_t mid, uint64_t last)
{
    uint64_t lcount = mid - first + 1;
    uint64_t ucount = last - mid;
    struct item *left = a + first;
    struct item *right = a + mid + 1;
    uint64_t i = 0, j = 0, k = 0;
    while (i < lcount && j < ucount) {
        if (key_le(kt, left[i].key, right[j].key))
            scratch[k++] = left[i++];
        else
            scratch[k++] = right[j++];
    }
    while (i < lcount)
        scratch[k++] = left[i++];
    while (j < ucount)
        scratch[k++] = right[j++];
    memcpy(a + first, scratch, (size_t)(lcount + ucount) * sizeof(struct item));
}

/* Figure 3: merge_sort(list, first, last) on the inclusive range. */
static void merge_sort(int kt, struct item *a, struct item *scratch, uint64_t first, uint64_t last)
{
    if (first >= last)
        return;
    uint64_t mid = first + (last - first) / 2;
    merge_sort(kt, a, scratch, first, mid);
    merge_sort(kt, a, scratch, mid + 1, last);
    merge_adjacent(kt, a, scratch, first, mid, last);
}

/* Sort n items in place (n may be 0). */
static int sort_items(int kt, struct item *a, uint64_t n)
{
    if (n < 2)
        return 0;
    struct item *scratch = (struct item *)malloc(n * sizeof(struct item));
    if (!scratch)
        return -3;
    merge_sort(kt, a, scratch, 0, n - 1);
    free(scratch);
    return 0;
}

/* Merge two sorted item arrays a (na items, the earlier run) and b (nb items,
 * the later run) into out; a's item first on ties. */
static void merge_two(int kt, const struct item *a, uint64_t na, const struct item *b, uint64_t nb,
                      struct item *out)
{
    uint64_t i = 0, j = 0, k = 0;
    while (i < na && j < nb) {
        if (key_le(kt, a[i].key, b[j].key))
            out[k++] = a[i++];
        else
            out[k++] = b[j++];
    }
    while (i < na)
        out[k++] = a[i++];
    while (j < nb)
        out[k++] = b[j++];
}

static int run_is_sorted(int kt, const struct item *a, uint64_t n)
{
    for (uint64_t i = 1; i < n; i++)
        if (key_lt(kt, a[i].key, a[i - 1].key))
            return 0;
    return 1;
}

/* Section 3.2.2: the master merges all the sorted sub-lists into one sorted
 * list.  Read here as the master folding the runs in order into its result:
 * result = merge(result, run_r) for r = 0, 1, ..., with the accumulated
 * (earlier) items first on ties.  a holds the runs back to back; off has
 * nruns + 1 entries.  Returns -2 if a run is not sorted. */
static int master_merge(int kt, struct item *a, const uint64_t *off, uint64_t nruns)
{
    uint64_t n = off[nruns];
    for (uint64_t r = 0; r < nruns; r++)
        if (!run_is_sorted(kt, a + off[r], off[r + 1] - off[r]))
            return -2;
    if (n == 0)
        return 0;
    struct item *acc = (struct item *)malloc(n * sizeof(struct item));
    struct item *tmp = (struct item *)malloc(n * sizeof(struct item));
    if (!acc || !tmp) {
        free(acc);
        free(tmp);
        return -3;
    }
    uint64_t have = 0;
    for (uint64_t r = 0; r < nruns; r++) {
        uint64_t len = off[r + 1] - off[r];
        merge_two(kt, acc, have, a + off[r], len, tmp);
        have += len;
        memcpy(acc, tmp, (size_t)have * sizeof(struct item));
    }
    memcpy(a, acc, (size_t)n * sizeof(struct item));
    free(acc);
    free(tmp);
    return 0;
}

static int offsets_ok(const uint64_t *off, uint64_t nseg, uint64_t n_total)
{
    if (off[0] != 0 || off[nseg] != n_total)
        return 0;
    for (uint64_t s = 0; s < nseg; s++)
        if (off[s + 1] < off[s])
            return 0;
    return 1;
}

/* Figure 1, scatter phase: the partition size is s = n/p.  Read for any n and
 * p >= 1 as part i = [floor(i*n/p), floor((i+1)*n/p)); when p divides n every
 * part has exactly s items, as in all of the paper's runs. */
static uint64_t part_begin(uint64_t n, uint64_t p, uint64_t i)
{
    return (uint64_t)(((unsigned __int128)i * n) / p);
}

/* ======================================================================== */
/* Exported entry points.  Return 0 on success, -1 for bad arguments, -2 for
 * a violated precondition (unsorted run, bad offsets), -3 for out of memory. */

/* The stable ascending sort of n keys (values optional, may be NULL). */
int oracle_sort(int kt, const void *keys_in, const uint32_t *vals_in, void *keys_out,
                uint32_t *vals_out, uint64_t n)
{
    if (!valid_kt(kt) || (n && (!keys_in || !keys_out)))
        return -1;
    struct item *a = read_items(kt, keys_in, vals_in, n);
    if (!a)
        return -3;
    int rc = sort_items(kt, a, n);
    if (rc == 0)
        write_items(kt, a, n, keys_out, vals_out);
    free(a);
    return rc;
}

/* Each segment [off[s], off[s+1]) sorted on its own; nothing crosses a
 * segment boundary.  Segments may be empty. */
int oracle_sort_segmented(int kt, const void *keys_in, const uint32_t *vals_in, void *keys_out,
                          uint32_t *vals_out, const uint64_t *off, uint64_t nseg)
{
    if (!valid_kt(kt) || !off)
        return -1;
    uint64_t n = off[nseg];
    if (n && (!keys_in || !keys_out))
        return -1;
    if (!offsets_ok(off, nseg, n))
        return -2;
    struct item *a = read_items(kt, keys_in, vals_in, n);
    if (!a)
        return -3;
    int rc = 0;
    for (uint64_t s = 0; s < nseg && rc == 0; s++)
        rc = sort_items(kt, a + off[s], off[s + 1] - off[s]);
    if (rc == 0)
        write_items(kt, a, n, keys_out, vals_out);
    free(a);
    return rc;
}

/* The merge phase: nruns adjacent sorted runs, combined by the master merge of
 * Section 3.2.2.  The result is the stable sort of the concatenation. */
int oracle_merge_runs(int kt, const void *keys_in, const uint32_t *vals_in, void *keys_out,
                      uint32_t *vals_out, const uint64_t *off, uint64_t nruns)
{
    if (!valid_kt(kt) || !off || nruns == 0)
        return -1;
    uint64_t n = off[nruns];
    if (n && (!keys_in || !keys_out))
        return -1;
    if (!offsets_ok(off, nruns, n))
        return -2;
    struct item *a = read_items(kt, keys_in, vals_in, n);
    if (!a)
        return -3;
    int rc = master_merge(kt, a, off, nruns);
    if (rc == 0)
        write_items(kt, a, n, keys_out, vals_out);
    free(a);
    return rc;
}

/* The whole method of Figure 1 with the master merge of Section 3.2.2:
 * partition into p parts, sort every part with Figure 3, merge at the master. */
int oracle_paper_method(int kt, const void *keys_in, const uint32_t *vals_in, void *keys_out,
                        uint32_t *vals_out, uint64_t n, uint64_t p)
{
    if (!valid_kt(kt) || p == 0 || (n && (!keys_in || !keys_out)))
        return -1;
    uint64_t *off = (uint64_t *)malloc((size_t)(p + 1) * sizeof(uint64_t));
    struct item *a = read_items(kt, keys_in, vals_in, n);
    if (!off || !a) {
        free(off);
        free(a);
        return -3;
    }
    for (uint64_t i = 0; i <= p; i++)
        off[i] = part_begin(n, p, i);
    int rc = 0;
    for (uint64_t i = 0; i < p && rc == 0; i++) /* sorting phase */
        rc = sort_items(kt, a + off[i], off[i + 1] - off[i]);
    if (rc == 0) /* merge phase */
        rc = master_merge(kt, a, off, p);
    if (rc == 0)
        write_items(kt, a, n, keys_out, vals_out);
    free(off);
    free(a);
    return rc;
}

/* Figure 1's merge phase read as odd/even transposition merge-split: p phases;
 * in an even phase the pairs are (0,1), (2,3), ..., in an odd phase (1,2),
 * (3,4), ...; each pair merges its two sorted parts (lower part first on ties)
 * and the lower process keeps the first |lower| items, the upper process the
 * rest, so every process keeps its own item count.  An unpaired process idles
 * for the phase.  Parts are first sorted as in the sorting phase.
 * The schedule needs equal parts (every run in the paper has p dividing n):
 * with unequal or empty parts, count-preserving exchanges cannot carry items
 * across, so p must divide n here (otherwise -2). */
int oracle_merge_split(int kt, const void *keys_in, const uint32_t *vals_in, void *keys_out,
                       uint32_t *vals_out, uint64_t n, uint64_t p)
{
    if (!valid_kt(kt) || p == 0 || (n && (!keys_in || !keys_out)))
        return -1;
    if (n % p != 0)
        return -2;
    uint64_t *off = (uint64_t *)malloc((size_t)(p + 1) * sizeof(uint64_t));
    struct item *a = read_items(kt, keys_in, vals_in, n);
    struct item *sorted_list = (struct item *)malloc((n ? n : 1) * sizeof(struct item));
    if (!off || !a || !sorted_list) {
        free(off);
        free(a);
        free(sorted_list);
        return -3;
    }
    for (uint64_t i = 0; i <= p; i++)
        off[i] = part_begin(n, p, i);
    int rc = 0;
    for (uint64_t i = 0; i < p && rc == 0; i++)
        rc = sort_items(kt, a + off[i], off[i + 1] - off[i]);
    for (uint64_t step = 0; step < p && rc == 0; step++) {
        for (uint64_t id = step % 2; id + 1 < p; id += 2) {
            uint64_t nlo = off[id + 1] - off[id];
            uint64_t nhi = off[id + 2] - off[id + 1];
            merge_two(kt, a + off[id], nlo, a + off[id + 1], nhi, sorted_list);
            /* the lower process keeps the first half, the upper the second */
            memcpy(a + off[id], sorted_list, (size_t)(nlo + nhi) * sizeof(struct item));
        }
    }
    if (rc == 0)
        write_items(kt, a, n, keys_out, vals_out);
    free(off);
    free(a);
    free(sorted_list);
    return rc;
}

/* Figure 2: bubble sort with adjacent exchanges when the left item is strictly
 * greater (so equal items never pass each other).  O(n^2): tiny inputs only. */
int oracle_bubble(int kt, const void *keys_in, const uint32_t *vals_in, void *keys_out,
                  uint32_t *vals_out, uint64_t n)
{
    if (!valid_kt(kt) || (n && (!keys_in || !keys_out)))
        return -1;
    struct item *a = read_items(kt, keys_in, vals_in, n);
    if (!a)
        return -3;
    for (int64_t i = (int64_t)n - 2; i >= 0; i--) {
        for (int64_t j = 0; j <= i; j++) {
            if (key_lt(kt, a[j + 1].key, a[j].key)) {
                struct item temp = a[j];
                a[j] = a[j + 1];
                a[j + 1] = temp;
            }
        }
    }
    write_items(kt, a, n, keys_out, vals_out);
    free(a);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The method with threads standing in for MPI processes (Figure 1 with the
 * Section 3.2.2 master merge): p parts, each sorted by Figure 3 on its own
 * thread, then the master merge on the calling thread.  Used only to time the
 * CPU baseline. */
struct part_job {
    int kt;
    struct item *a;
    uint64_t n;
    int rc;
};

static void *part_worker(void *arg)
{
    struct part_job *job = (struct part_job *)arg;
    job->rc = sort_items(job->kt, job->a, job->n);
    return NULL;
}

int oracle_paper_method_threads(int kt, const void *keys_in, const uint32_t *vals_in,
                                void *keys_out, uint32_t *vals_out, uint64_t n, uint64_t p)
{
    if (!valid_kt(kt) || p == 0 || p > 4096 || (n && (!keys_in || !keys_out)))
        return -1;
    uint64_t *off = (uint64_t *)malloc((size_t)(p + 1) * sizeof(uint64_t));
    struct item *a = read_items(kt, keys_in, vals_in, n);
    pthread_t *th = (pthread_t *)malloc((size_t)p * sizeof(pthread_t));
    struct part_job *jobs = (struct part_job *)malloc((size_t)p * sizeof(struct part_job));
    int rc = 0;
    if (!off || !a || !th || !jobs) {
        rc = -3;
        goto done;
    }
    for (uint64_t i = 0; i <= p; i++)
        off[i] = part_begin(n, p, i);
    for (uint64_t i = 0; i < p; i++) {
        jobs[i].kt = kt;
        jobs[i].a = a + off[i];
        jobs[i].n = off[i + 1] - off[i];
        jobs[i].rc = 0;
        if (pthread_create(&th[i], NULL, part_worker, &jobs[i]) != 0) {
            jobs[i].rc = -3;
            th[i] = 0;
        }
    }
    for (uint64_t i = 0; i < p; i++) {
        if (th[i])
            pthread_join(th[i], NULL);
        if (jobs[i].rc)
            rc = jobs[i].rc;
    }
    if (rc == 0)
        rc = master_merge(kt, a, off, p);
    if (rc == 0)
        write_items(kt, a, n, keys_out, vals_out);
done:
    free(off);
    free(a);
    free(th);
    free(jobs);
    return rc;
}

/* Bytes per key for a key type code, or 0 if the code is unknown. */
int oracle_key_bytes(int kt) { return valid_kt(kt) ? (int)key_bytes(kt) : 0; }
