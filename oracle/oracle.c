/*
 * CPU ORACLE — test infrastructure only.
 *
 * Plain, slow, single-threaded C that states what the GPU merge sort must
 * compute.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark load this library; the product path never does.  Nothing in
 * here is shared with the HIP sources: the networks are generated from their
 * textbook definition at run time, comparisons use the plain dtype order, and
 * every sort follows the paper's top-down algorithm, its recursion kept on an
 * explicit stack.
 *
 * Paper: Aly, Jensen, ElAarag, "Improving Merge Sort and Quick Sort
 * Performance by Utilizing AlphaDev's Sorting Networks as Base Cases",
 * ACMSE 2025 (arXiv 2503.05934).
 *
 *   - orc_sort(ORC_MS, ...)      Algorithm 1 (merge sort with network base
 *                                cases); with an empty network set it is the
 *                                classical merge sort the paper measures
 *                                against (Sec. 3, Eq. 1).
 *   - orc_sort(ORC_QS, ...)      Algorithm 2 (quick sort with network base
 *                                cases), median-of-three pivots and Hoare
 *                                partitioning (Sec. 3); with an empty set it
 *                                is the classical quick sort.
 *   - orc_config_mask            the network sets of Table 3.
 *   - orc_network                the fixed sorting networks for sizes 2..8
 *                                (the role AlphaDev's networks play, Sec. 1/3),
 *                                built here from Batcher's odd-even merge sort.
 *   - orc_segmented_sort         the above per CSR segment.
 *   - orc_gather_backward        gradient of a sort: grad_in[perm[i]] =
 *                                grad_out[i] (not in the paper; definition).
 *
 * Readings of the paper taken here (the paper is silent on them):
 *   - key types: uint32, int32, float32; ascending order.
 *   - float32 order: IEEE "<", so -0 and +0 tie; every NaN sorts after +inf
 *     and all NaNs tie with each other.
 *   - Merge takes from the left run on ties (stable).
 *   - "stable" sorts compare (key, original position) so that a network, which
 *     is not stable on keys alone, still yields the stable order.
 *   - the median-of-three step orders the first, middle and last records in
 *     place and pivots on the middle one; the partition is Hoare's 1962
 *     scheme around that pivot value.
 *   - VarSortK (Table 3) handles every size up to K, so its set is {2..K}.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_U32 0
#define ORC_I32 1
#define ORC_F32 2

#define ORC_MS 0 /* Algorithm 1 (merge sort) */
#define ORC_QS 1 /* Algorithm 2 (quick sort) */

#define ORC_MAX_NET 8
#define ORC_MAX_CMP 32

/* One element being sorted: the key bits, its payload, and its original
 * position (used only to break ties when a stable order is asked for). */
typedef struct {
    uint32_t key;
    uint32_t val;
    uint32_t pos;
} rec_t;

typedef struct {
    int dtype;
    int stable;
} order_t;

/* ---------------------------------------------------------------- order --- */

static float bits_to_f32(uint32_t b) {
    float f;
    memcpy(&f, &b, sizeof f);
    return f;
}

/* a < b in the plain order of the dtype. */
static int key_less(int dtype, uint32_t a, uint32_t b) {
    if (dtype == ORC_U32) return a < b;
    if (dtype == ORC_I32) return (int32_t)a < (int32_t)b;
    {
        float fa = bits_to_f32(a), fb = bits_to_f32(b);
        if (isnan(fa)) return 0;         /* NaN is never below anything */
        if (isnan(fb)) return 1;         /* every number is below NaN    */
        return fa < fb;                  /* IEEE: -0 < +0 is false       */
    }
}

static int rec_less(const order_t* o, const rec_t* a, const rec_t* b) {
    if (key_less(o->dtype, a->key, b->key)) return 1;
    if (key_less(o->dtype, b->key, a->key)) return 0;
    return o->stable && a->pos < b->pos;
}

/* ------------------------------------------------------------- networks --- */
/*
 * Batcher's odd-even merge sort for 8 wires, from its recursive definition
 * (Batcher 1968; Knuth, TAOCP vol. 3, Sec. 5.3.4).  The network for n < 8
 * wires keeps the comparators whose wires are both below n (the others would
 * only ever see +infinity on their upper wire), and then drops any comparator
 * that never exchanges for any of the 2^n zero-one inputs.
 */
static int g_net_ready = 0;
static int g_net_len[ORC_MAX_NET + 1];
static int g_net[ORC_MAX_NET + 1][ORC_MAX_CMP][2];

static int g_full_len;
static int g_full[ORC_MAX_CMP][2];

static void batcher_add(int i, int j) {
    g_full[g_full_len][0] = i;
    g_full[g_full_len][1] = j;
    g_full_len++;
}

/* merge the two sorted halves of wires lo, lo+r, lo+2r, ... (n wires) */
static void batcher_merge(int lo, int n, int r) {
    int step = r * 2;
    if (step < n) {
        batcher_merge(lo, n, step);       /* even subsequence */
        batcher_merge(lo + r, n, step);   /* odd subsequence  */
        for (int i = lo + r; i + r < lo + n; i += step) batcher_add(i, i + r);
    } else {
        batcher_add(lo, lo + r);
    }
}

static void batcher_sort(int lo, int n) {
    if (n > 1) {
        int m = n / 2;
        batcher_sort(lo, m);
        batcher_sort(lo + m, m);
        batcher_merge(lo, n, 1);
    }
}

static void build_networks(void) {
    if (g_net_ready) return;
    g_full_len = 0;
    batcher_sort(0, ORC_MAX_NET);
    for (int n = 0; n <= ORC_MAX_NET; n++) {
        int kept[ORC_MAX_CMP][2], nk = 0;
        for (int c = 0; c < g_full_len; c++)
            if (g_full[c][1] < n) {
                kept[nk][0] = g_full[c][0];
                kept[nk][1] = g_full[c][1];
                nk++;
            }
        /* a comparator is useful if it exchanges for some 0-1 input */
        int useful[ORC_MAX_CMP] = {0};
        for (uint32_t in = 0; in < (1u << n); in++) {
            int w[ORC_MAX_NET];
            for (int b = 0; b < n; b++) w[b] = (in >> b) & 1;
            for (int c = 0; c < nk; c++) {
                int i = kept[c][0], j = kept[c][1];
                if (w[j] < w[i]) {
                    int t = w[i];
                    w[i] = w[j];
                    w[j] = t;
                    useful[c] = 1;
                }
            }
        }
        g_net_len[n] = 0;
        for (int c = 0; c < nk; c++)
            if (useful[c]) {
                g_net[n][g_net_len[n]][0] = kept[c][0];
                g_net[n][g_net_len[n]][1] = kept[c][1];
                g_net_len[n]++;
            }
    }
    g_net_ready = 1;
}

/* Writes the n-wire network as (i, j) pairs, i < j, in application order.
 * Returns the number of comparators, or -1 for n outside 0..8. */
int orc_network(int n, int* pairs_out) {
    if (n < 0 || n > ORC_MAX_NET) return -1;
    build_networks();
    for (int c = 0; c < g_net_len[n]; c++) {
        pairs_out[2 * c] = g_net[n][c][0];
        pairs_out[2 * c + 1] = g_net[n][c][1];
    }
    return g_net_len[n];
}

/* The network base case of Algorithms 1 and 2: sorts a[0..n-1] with the
 * n-input network. */
static void apply_network(const order_t* o, rec_t* a, int n) {
    build_networks();
    for (int c = 0; c < g_net_len[n]; c++) {
        rec_t* x = &a[g_net[n][c][0]];
        rec_t* y = &a[g_net[n][c][1]];
        if (rec_less(o, y, x)) {
            rec_t t = *x;
            *x = *y;
            *y = t;
        }
    }
}

/* Applies the n-network to each of `count` consecutive n-tuples of keys.
 * perm (optional) receives, per tuple, the tuple-local position each output
 * came from.  Used to test the networks exhaustively. */
int orc_apply_network_batch(int n, int dtype, int stable, uint32_t* keys,
                            uint32_t* perm, int64_t count) {
    if (n < 0 || n > ORC_MAX_NET || count < 0) return -1;
    order_t o = {dtype, stable};
    rec_t r[ORC_MAX_NET];
    for (int64_t t = 0; t < count; t++) {
        for (int i = 0; i < n; i++) {
            r[i].key = keys[t * n + i];
            r[i].val = (uint32_t)i;
            r[i].pos = (uint32_t)i;
        }
        apply_network(&o, r, n);
        for (int i = 0; i < n; i++) {
            keys[t * n + i] = r[i].key;
            if (perm) perm[t * n + i] = r[i].val;
        }
    }
    return 0;
}

/* --------------------------------------------------------- configurations */
/* Table 3: which network sizes each configuration enables (bit k = size k). */
int64_t orc_config_mask(const char* name) {
    static const struct {
        const char* name;
        uint32_t mask;
    } table[] = {
        {"PowerOf2", (1u << 4) | (1u << 8)},
        {"Even", (1u << 4) | (1u << 6) | (1u << 8)},
        {"Odd", (1u << 3) | (1u << 5) | (1u << 7)},
        {"3", (1u << 3)},
        {"3To4", (1u << 3) | (1u << 4)},
        {"3To5", (1u << 3) | (1u << 4) | (1u << 5)},
        {"3To8", 0x1f8u},
        {"6To8", (1u << 6) | (1u << 7) | (1u << 8)},
        {"VarSort3", 0x0cu},
        {"VarSort4", 0x1cu},
        {"VarSort5", 0x3cu},
        {"Classical", 0u},
    };
    for (size_t i = 0; i < sizeof table / sizeof table[0]; i++)
        if (strcmp(name, table[i].name) == 0) return table[i].mask;
    return -1;
}

/* -------------------------------------------------------- shared pieces --- */

/* Ranges are half-open: `count` records starting at index `start`. */
typedef struct {
    int64_t start;
    int64_t count;
    int merge_pending; /* merge sort only: both halves are sorted, merge them */
} range_t;

/* Deep enough for any count below 2^63: every split at least halves the
 * larger part, and a range waits on the stack with at most one sibling and
 * its own merge marker per level. */
#define ORC_STACK 256

/* The base case of Sec. 3: a range is handed to a sorting network exactly
 * when its size is one of the sizes the configuration enables (Table 3). */
static int network_takes(uint32_t netmask, int64_t count) {
    return count >= 0 && count <= ORC_MAX_NET && ((netmask >> count) & 1u) != 0;
}

/* ----------------------------------------------------------- merge sort --- */

typedef struct {
    order_t ord;
    uint32_t netmask;
    rec_t* scratch;
    int64_t* leaf_hist; /* optional: elements handled by each network size */
} ms_ctx;

/* The Merge step of Algorithm 1: the two sorted neighbours a[start ..
 * start+nl) and a[start+nl .. start+total) become one sorted range.  An
 * element of the right neighbour goes first only when it is strictly
 * smaller, so equal elements keep their left-to-right order. */
static void merge_neighbours(ms_ctx* c, rec_t* a, int64_t start, int64_t nl, int64_t total) {
    const rec_t* left = a + start;
    const rec_t* right = a + start + nl;
    const int64_t nr = total - nl;
    int64_t li = 0, ri = 0;
    for (int64_t out = 0; out < total; out++) {
        int from_right;
        if (li == nl)
            from_right = 1;
        else if (ri == nr)
            from_right = 0;
        else
            from_right = rec_less(&c->ord, &right[ri], &left[li]);
        c->scratch[out] = from_right ? right[ri++] : left[li++];
    }
    memcpy(a + start, c->scratch, (size_t)total * sizeof(rec_t));
}

/* Algorithm 1 (Sec. 3), top-down merge sort with network base cases, driven
 * by an explicit stack instead of recursion.  A range whose size the
 * configuration enables goes to that network.  Any other range of two or
 * more records is cut at its midpoint, the left part taking the extra record
 * of an odd count (the split the paper's midpoint index gives); once both
 * parts are sorted they are merged.  Ranges of 0 or 1 records are done. */
static void network_merge_sort(ms_ctx* c, rec_t* a, int64_t n) {
    range_t stack[ORC_STACK];
    int top = 0;
    stack[top++] = (range_t){0, n, 0};
    while (top > 0) {
        range_t r = stack[--top];
        const int64_t nl = r.count - r.count / 2;
        if (r.merge_pending) {
            merge_neighbours(c, a, r.start, nl, r.count);
        } else if (network_takes(c->netmask, r.count)) {
            apply_network(&c->ord, a + r.start, (int)r.count);
            if (c->leaf_hist) c->leaf_hist[r.count] += r.count;
        } else if (r.count >= 2) {
            /* the merge runs after both parts, which sit above it */
            stack[top++] = (range_t){r.start, r.count, 1};
            stack[top++] = (range_t){r.start + nl, r.count - nl, 0};
            stack[top++] = (range_t){r.start, nl, 0};
        }
    }
}

/* ----------------------------------------------------------- quick sort --- */

static void swap_rec(rec_t* x, rec_t* y) {
    rec_t t = *x;
    *x = *y;
    *y = t;
}

/* Median-of-three pivot choice (Algorithm 2): the first, middle and last
 * records of the range are put in order among themselves, and the middle
 * one, now their median, is the pivot.  Returns a copy of it. */
static rec_t pivot_of_three(const order_t* o, rec_t* a, int64_t first, int64_t last) {
    const int64_t middle = first + (last - first) / 2;
    if (rec_less(o, &a[middle], &a[first])) swap_rec(&a[middle], &a[first]);
    if (rec_less(o, &a[last], &a[first])) swap_rec(&a[last], &a[first]);
    if (rec_less(o, &a[last], &a[middle])) swap_rec(&a[last], &a[middle]);
    return a[middle];
}

/* Hoare's partition (Algorithm 2; Hoare 1962): two scans move towards each
 * other, the left one stopping at a record not below the pivot, the right
 * one at a record not above it; such a pair is exchanged and both scans step
 * on.  When they meet or cross, every record up to the right scan's position
 * is no greater than the pivot and every record after it no smaller.
 * Returns that position, which lies in [first, last). */
static int64_t hoare_split(const order_t* o, rec_t* a, int64_t first, int64_t last,
                           const rec_t* pivot) {
    int64_t up = first, down = last;
    for (;;) {
        while (rec_less(o, &a[up], pivot)) up++;
        while (rec_less(o, pivot, &a[down])) down--;
        if (up >= down) return down;
        swap_rec(&a[up], &a[down]);
        up++;
        down--;
    }
}

/* Algorithm 2 (Sec. 3), quick sort with network base cases, driven by an
 * explicit stack.  A range whose size the configuration enables goes to that
 * network; any other range of two or more records is split by Hoare's
 * partition around its median-of-three pivot, and both parts are sorted the
 * same way. */
static void network_quick_sort(const order_t* o, uint32_t netmask, rec_t* a, int64_t n) {
    range_t stack[ORC_STACK];
    int top = 0;
    stack[top++] = (range_t){0, n, 0};
    while (top > 0) {
        range_t r = stack[--top];
        if (network_takes(netmask, r.count)) {
            apply_network(o, a + r.start, (int)r.count);
        } else if (r.count >= 2) {
            const int64_t last = r.start + r.count - 1;
            const rec_t pivot = pivot_of_three(o, a, r.start, last);
            const int64_t cut = hoare_split(o, a, r.start, last, &pivot);
            /* smaller part on top: the stack stays logarithmic */
            const range_t lo = {r.start, cut - r.start + 1, 0};
            const range_t hi = {cut + 1, last - cut, 0};
            if (lo.count < hi.count) {
                stack[top++] = hi;
                stack[top++] = lo;
            } else {
                stack[top++] = lo;
                stack[top++] = hi;
            }
        }
    }
}

/* ------------------------------------------------------------- drivers --- */

static int sort_records(int algo, const order_t* o, uint32_t netmask, rec_t* r,
                        int64_t n, rec_t* scratch, int64_t* leaf_hist) {
    if (n <= 0) return 0;
    if (algo == ORC_MS) {
        ms_ctx c = {*o, netmask, scratch, leaf_hist};
        network_merge_sort(&c, r, n);
    } else {
        network_quick_sort(o, netmask, r, n);
    }
    return 0;
}

static int check_args(int algo, int dtype, uint32_t netmask) {
    if (algo != ORC_MS && algo != ORC_QS) return -4;
    if (dtype != ORC_U32 && dtype != ORC_I32 && dtype != ORC_F32) return -3;
    if (netmask & ~0x1feu) return -4; /* sizes 1..8 only */
    return 0;
}

/*
 * Sorts keys[0..n-1] (bits of dtype) in place, ascending.  If vals is not
 * NULL it is permuted along with the keys.  If perm is not NULL it receives
 * the original position of each output element.  stable != 0 orders equal
 * keys by original position.  Returns 0, or a negative code on bad input.
 */
int orc_sort(int algo, int dtype, uint32_t netmask, int stable, uint32_t* keys,
             uint32_t* vals, uint32_t* perm, int64_t n) {
    int rc = check_args(algo, dtype, netmask);
    if (rc) return rc;
    if (n < 0 || n > 0xffffffffLL) return -2;
    if (n == 0) return 0;
    if (!keys) return -1;
    order_t o = {dtype, stable};
    rec_t* r = (rec_t*)malloc((size_t)n * sizeof(rec_t));
    rec_t* s = algo == ORC_MS ? (rec_t*)malloc((size_t)n * sizeof(rec_t)) : NULL;
    if (!r || (algo == ORC_MS && !s)) {
        free(r);
        free(s);
        return -7;
    }
    for (int64_t i = 0; i < n; i++) {
        r[i].key = keys[i];
        r[i].val = vals ? vals[i] : (uint32_t)i;
        r[i].pos = (uint32_t)i;
    }
    sort_records(algo, &o, netmask, r, n, s, NULL);
    for (int64_t i = 0; i < n; i++) {
        keys[i] = r[i].key;
        if (vals) vals[i] = r[i].val;
        if (perm) perm[i] = r[i].pos;
    }
    free(r);
    free(s);
    return 0;
}

/*
 * Per-segment sort.  Segment s is keys[offsets[s] .. offsets[s+1]-1].
 * perm (optional) receives the segment-local original position of each
 * output element.  offsets must start at 0, never decrease and end at the
 * total length; -2 otherwise.
 */
int orc_segmented_sort(int algo, int dtype, uint32_t netmask, int stable,
                       uint32_t* keys, uint32_t* vals, uint32_t* perm,
                       const uint32_t* offsets, int64_t num_segments) {
    int rc = check_args(algo, dtype, netmask);
    if (rc) return rc;
    if (num_segments < 0) return -2;
    if (num_segments == 0) return 0;
    if (!offsets) return -1;
    if (offsets[0] != 0) return -2;
    int64_t longest = 0;
    for (int64_t s = 0; s < num_segments; s++) {
        if (offsets[s + 1] < offsets[s]) return -2;
        int64_t len = (int64_t)offsets[s + 1] - offsets[s];
        if (len > longest) longest = len;
    }
    if (longest == 0) return 0;
    if (!keys) return -1;
    order_t o = {dtype, stable};
    rec_t* r = (rec_t*)malloc((size_t)longest * sizeof(rec_t));
    rec_t* sc = (rec_t*)malloc((size_t)longest * sizeof(rec_t));
    if (!r || !sc) {
        free(r);
        free(sc);
        return -7;
    }
    for (int64_t s = 0; s < num_segments; s++) {
        int64_t b = offsets[s], len = (int64_t)offsets[s + 1] - offsets[s];
        for (int64_t i = 0; i < len; i++) {
            r[i].key = keys[b + i];
            r[i].val = vals ? vals[b + i] : (uint32_t)i;
            r[i].pos = (uint32_t)i;
        }
        sort_records(algo, &o, netmask, r, len, sc, NULL);
        for (int64_t i = 0; i < len; i++) {
            keys[b + i] = r[i].key;
            if (vals) vals[b + i] = r[i].val;
            if (perm) perm[b + i] = r[i].pos;
        }
    }
    free(r);
    free(sc);
    return 0;
}

/*
 * Counts, for Algorithm 1 on an array of n elements, how many elements end
 * in a network of each size (hist[0..8]).  Shows which leaves a
 * configuration reaches for a given n; the data do not matter.
 */
int orc_alg1_leaf_histogram(int64_t n, uint32_t netmask, int64_t* hist) {
    if (n < 0 || !hist) return -2;
    for (int k = 0; k <= ORC_MAX_NET; k++) hist[k] = 0;
    if (n == 0) return 0;
    order_t o = {ORC_U32, 0};
    rec_t* r = (rec_t*)calloc((size_t)n, sizeof(rec_t));
    rec_t* s = (rec_t*)malloc((size_t)n * sizeof(rec_t));
    if (!r || !s) {
        free(r);
        free(s);
        return -7;
    }
    sort_records(ORC_MS, &o, netmask, r, n, s, hist);
    free(r);
    free(s);
    return 0;
}

/*
 * Backward of y = sort(x) along each row: y[r][i] = x[r][perm[r][i]], so
 * d<g, y>/dx[r][perm[r][i]] = g[r][i].  Entries of perm outside [0, cols)
 * make the call fail with -2 before anything is written.
 */
int orc_gather_backward(const float* grad_out, const int32_t* perm, float* grad_in,
                        int64_t rows, int64_t cols) {
    if (rows < 0 || cols < 0) return -2;
    if (rows * cols == 0) return 0;
    if (!grad_out || !perm || !grad_in) return -1;
    for (int64_t e = 0; e < rows * cols; e++)
        if (perm[e] < 0 || perm[e] >= cols) return -2;
    for (int64_t r = 0; r < rows; r++)
        for (int64_t i = 0; i < cols; i++)
            grad_in[r * cols + perm[r * cols + i]] = grad_out[r * cols + i];
    return 0;
}

/*
 * Rank check for one output value v of a sort of keys[0..n-1]: *less counts
 * keys ordered strictly before v, *less_equal those not ordered after it.
 * y is the sorted output iff less(y[i]) <= i < less_equal(y[i]) for every i,
 * so any sample of positions can be checked one by one at any size.
 */
int orc_rank_bounds(int dtype, const uint32_t* keys, int64_t n, uint32_t v, int64_t* less,
                    int64_t* less_equal) {
    if (dtype != ORC_U32 && dtype != ORC_I32 && dtype != ORC_F32) return -3;
    if (n < 0) return -2;
    if ((n > 0 && !keys) || !less || !less_equal) return -1;
    int64_t lt = 0, le = 0;
    for (int64_t i = 0; i < n; i++) {
        if (key_less(dtype, keys[i], v)) lt++;
        if (!key_less(dtype, v, keys[i])) le++;
    }
    *less = lt;
    *less_equal = le;
    return 0;
}
