/*
 * CPU oracle for unsorted top-k selection (Hübschle-Schneider, Sanders, Müller,
 * "Communication Efficient Algorithms for Top-k Selection Problems").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this file.  It shares no code with the
 * GPU library: it uses plain comparisons on the original keys (no bit
 * encodings of the key order), a library sort, and straight loops.
 *
 * Contents
 *   - the key order with the (value, object) tie rule          (§2, Preliminaries)
 *   - select by full sort                      ("plain" oracle, §4 problem statement)
 *   - select by brute-force rank counting      (pins the plain oracle on tiny inputs)
 *   - select by a sort of 64-bit composites    (the same result; the form the benchmark
 *                                               times, on one thread or several)
 *   - an O(n) checker of a claimed result      (invariants of the selection problem)
 *   - Philox4x32-10                             (Salmon et al., SC'11, published definition)
 *   - Bernoulli sampling with geometric skips  (§2, "Bernoulli sampling")
 *   - pivot ranks around k|S|/n ± Δ            (§2, distributed FR-selection; §4.1 proof)
 *   - the rank of an object in the unique order  (§2 order, §4 problem statement): the
 *                                               counts |a| and |b| of a round of the
 *                                               Algorithm of §2 are rank differences
 *
 * All integer results are exact.  The only floating point is inside the skip
 * computation of the sampler (fp64 log), which decides sample positions only.
 */
#define _GNU_SOURCE
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Key order.  §2 makes every value unique by pairing it with its object; the
 * object here is the 0-based position in the input.  Floats: all NaNs compare
 * equal to each other and above every number; -0.0 equals +0.0 (IEEE `<`).
 * `largest` reverses the value order only; ties stay by ascending position. */

typedef struct {
    const void *keys;
    int is_f32;
    int largest;
} orc_order;

static int val_less_raw(const orc_order *o, uint64_t i, uint64_t j)
{
    if (o->is_f32) {
        float a = ((const float *)o->keys)[i];
        float b = ((const float *)o->keys)[j];
        if (isnan(a)) return 0;
        if (isnan(b)) return 1;
        return a < b;
    } else {
        uint32_t a = ((const uint32_t *)o->keys)[i];
        uint32_t b = ((const uint32_t *)o->keys)[j];
        return a < b;
    }
}

/* less(x_i, x_j) in the selection order */
static int val_less(const orc_order *o, uint64_t i, uint64_t j)
{
    return o->largest ? val_less_raw(o, j, i) : val_less_raw(o, i, j);
}

/* i precedes j in the unique total order (value, then position) */
static int precedes(const orc_order *o, uint64_t i, uint64_t j)
{
    if (val_less(o, i, j)) return 1;
    if (val_less(o, j, i)) return 0;
    return i < j;
}

static int cmp_idx(const void *pa, const void *pb, void *ctx)
{
    const orc_order *o = (const orc_order *)ctx;
    uint32_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
    if (a == b) return 0;
    return precedes(o, a, b) ? -1 : 1;
}

int orc_precedes(const void *keys, int is_f32, int largest, uint32_t i, uint32_t j)
{
    orc_order o = {keys, is_f32, largest};
    return precedes(&o, i, j);
}

/* ------------------------------------------------------------------------ */
/* Plain oracle (§4: identify the elements of rank <= k).  Sort all positions
 * in the total order, keep the first k.  out_idx receives them in that order,
 * so out_idx[k-1] is the object of rank k. */
int orc_select_sort(const void *keys, int is_f32, uint64_t n, uint64_t k,
                    int largest, uint32_t *out_idx)
{
    if (n == 0 || k == 0 || k > n || n > 0xFFFFFFFFull) return -1;
    orc_order o = {keys, is_f32, largest};
    uint32_t *perm = (uint32_t *)malloc(n * sizeof(uint32_t));
    if (!perm) return -2;
    for (uint64_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
    qsort_r(perm, n, sizeof(uint32_t), cmp_idx, &o);
    memcpy(out_idx, perm, k * sizeof(uint32_t));
    free(perm);
    return 0;
}

/* Brute force: rank(i) = #{j : j precedes i}; i is selected iff rank(i) < k.
 * out_idx receives the selected positions in ascending position order;
 * *kth_idx the one of rank k.  O(n^2); meant for n of a few thousand. */
int orc_select_brute(const void *keys, int is_f32, uint64_t n, uint64_t k,
                     int largest, uint32_t *out_idx, uint32_t *kth_idx)
{
    if (n == 0 || k == 0 || k > n) return -1;
    orc_order o = {keys, is_f32, largest};
    uint64_t m = 0;
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t rank = 0;
        for (uint64_t j = 0; j < n; ++j)
            if (j != i && precedes(&o, j, i)) ++rank;
        if (rank < k) out_idx[m++] = (uint32_t)i;
        if (rank == k - 1) *kth_idx = (uint32_t)i;
    }
    return m == k ? 0 : -3;
}

/* ------------------------------------------------------------------------ */
/* The same selection by a sort of 64-bit composites (value order word << 32 |
 * position), whose unsigned order is the unique order of §2: the form the
 * benchmark times.  The value order word of a float is its IEEE bit pattern
 * made monotone: all NaNs map to the largest word, -0.0 to the word of +0.0,
 * negative numbers to the complement of their bits, the others to their bits
 * with the sign bit set.  `largest` complements the word (the position part
 * stays ascending).  With `threads` > 1 the composites are cut into that many
 * chunks, each sorted by its own thread, and the first k are merged. */
static uint32_t orc_value_word(const void *keys, int is_f32, uint64_t i, int largest)
{
    uint32_t b = ((const uint32_t *)keys)[i];
    uint32_t w;
    if (!is_f32) {
        w = b;
    } else {
        float f;
        memcpy(&f, &b, 4);
        if (isnan(f)) w = 0xFFFFFFFFu;
        else if (f == 0.0f) w = 0x80000000u;
        else if (b & 0x80000000u) w = ~b;
        else w = b | 0x80000000u;
    }
    return largest ? ~w : w;
}

static int cmp_u64(const void *pa, const void *pb)
{
    uint64_t a = *(const uint64_t *)pa, b = *(const uint64_t *)pb;
    return a < b ? -1 : a > b ? 1 : 0;
}

typedef struct {
    const void *keys;
    int is_f32, largest;
    uint64_t *c;
    uint64_t lo, hi;
} orc_chunk;

static void *orc_chunk_sort(void *arg)
{
    orc_chunk *ch = (orc_chunk *)arg;
    for (uint64_t i = ch->lo; i < ch->hi; ++i)
        ch->c[i] = ((uint64_t)orc_value_word(ch->keys, ch->is_f32, i, ch->largest) << 32) | i;
    qsort(ch->c + ch->lo, ch->hi - ch->lo, sizeof(uint64_t), cmp_u64);
    return NULL;
}

int orc_select_composite(const void *keys, int is_f32, uint64_t n, uint64_t k, int largest,
                         int threads, uint32_t *out_idx)
{
    if (n == 0 || k == 0 || k > n || n > 0xFFFFFFFFull || threads < 1) return -1;
    if ((uint64_t)threads > n) threads = (int)n;
    uint64_t *c = (uint64_t *)malloc(n * sizeof(uint64_t));
    orc_chunk *ch = (orc_chunk *)calloc((size_t)threads, sizeof(orc_chunk));
    pthread_t *th = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
    uint64_t *head = (uint64_t *)calloc((size_t)threads, sizeof(uint64_t));
    if (!c || !ch || !th || !head) { free(c); free(ch); free(th); free(head); return -2; }
    for (int t = 0; t < threads; ++t) {
        ch[t].keys = keys; ch[t].is_f32 = is_f32; ch[t].largest = largest; ch[t].c = c;
        ch[t].lo = n * (uint64_t)t / (uint64_t)threads;
        ch[t].hi = n * (uint64_t)(t + 1) / (uint64_t)threads;
    }
    int rc = 0;
    if (threads == 1) {
        orc_chunk_sort(&ch[0]);
    } else {
        int started = 0;
        for (; started < threads; ++started)
            if (pthread_create(&th[started], NULL, orc_chunk_sort, &ch[started]) != 0) break;
        for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
        if (started < threads) rc = -2;
    }
    /* merge the first k: repeatedly take the smallest chunk head */
    for (int t = 0; t < threads && rc == 0; ++t) head[t] = ch[t].lo;
    for (uint64_t m = 0; m < k && rc == 0; ++m) {
        int best = -1;
        for (int t = 0; t < threads; ++t)
            if (head[t] < ch[t].hi && (best < 0 || c[head[t]] < c[head[best]])) best = t;
        out_idx[m] = (uint32_t)c[head[best]];
        ++head[best];
    }
    free(c); free(ch); free(th); free(head);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* O(n) check of a claimed result (sel[0..k), kth_idx, kth_key_bits) against
 * the definition.  Returns 0 when every invariant holds, otherwise the number
 * of the first one that fails:
 *   1  an index is >= n or repeated
 *   2  kth_idx is not among the selected
 *   3  a selected element lies above the k-th value
 *   4  an unselected element lies below the k-th value
 *   5  counts: c_lt < k <= c_lt + c_eq and c_lt + (#selected ties) = k fail
 *   6  tie rule: a selected tie has a larger position than an unselected tie
 *   7  kth_idx is not the largest position among the selected ties
 *   8  kth_key_bits differ from the input's bits at kth_idx                 */
int orc_check(const void *keys, int is_f32, uint64_t n, uint64_t k, int largest,
              const uint32_t *sel, uint32_t kth_idx, uint32_t kth_key_bits)
{
    orc_order o = {keys, is_f32, largest};
    uint8_t *mark = (uint8_t *)calloc(n ? n : 1, 1);
    if (!mark) return -2;
    int rc = 0;
    for (uint64_t i = 0; i < k; ++i) {
        if (sel[i] >= n || mark[sel[i]]) { rc = 1; goto done; }
        mark[sel[i]] = 1;
    }
    if (kth_idx >= n || !mark[kth_idx]) { rc = 2; goto done; }
    uint64_t c_lt = 0, c_eq = 0, m_eq = 0;
    int64_t max_sel_tie = -1, min_unsel_tie = -1;
    for (uint64_t i = 0; i < n; ++i) {
        int below = val_less(&o, i, kth_idx);
        int above = val_less(&o, kth_idx, i);
        if (mark[i] && above) { rc = 3; goto done; }
        if (!mark[i] && below) { rc = 4; goto done; }
        if (below) ++c_lt;
        if (!below && !above) {
            ++c_eq;
            if (mark[i]) { ++m_eq; max_sel_tie = (int64_t)i; }
            else if (min_unsel_tie < 0) min_unsel_tie = (int64_t)i;
        }
    }
    if (!(c_lt < k && k <= c_lt + c_eq && c_lt + m_eq == k)) { rc = 5; goto done; }
    if (min_unsel_tie >= 0 && max_sel_tie > min_unsel_tie) { rc = 6; goto done; }
    if ((int64_t)kth_idx != max_sel_tie) { rc = 7; goto done; }
    {
        uint32_t bits;
        memcpy(&bits, (const char *)keys + 4 * (uint64_t)kth_idx, 4);
        if (bits != kth_key_bits) { rc = 8; goto done; }
    }
done:
    free(mark);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11).  Each round multiplies words 0 and 2
 * by fixed 32-bit constants and mixes the high halves with the other words and
 * the key; the key advances by the Weyl constants between rounds. */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint64_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = M0 * (uint64_t)c0;
        uint64_t p1 = M1 * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform number number `j` of stream (seed, tag, seg): counter (j/4, seg,
 * tag, 0), key (seed low, seed high), output word j%4, mapped to the open
 * interval (0,1) as (x + 1/2) / 2^32. */
static double uniform01(uint64_t seed, uint32_t tag, uint32_t seg, uint64_t j)
{
    uint32_t ctr[4] = {(uint32_t)(j >> 2), seg, tag, 0};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return ((double)out[j & 3] + 0.5) * (1.0 / 4294967296.0);
}

/* Bernoulli sample of positions 0..n-1 with probability rho (§2, "Bernoulli
 * sampling"): the gaps between sampled positions are geometric skip values,
 * drawn by inversion, skip = 1 + floor(ln U / ln(1 - rho)).
 * The n positions are cut into nseg equal segments of ceil(n/nseg); segment t
 * draws its skips from stream (seed, tag, t) starting just before its first
 * position (the geometric law is memoryless, so this is still one Bernoulli
 * sample) and keeps at most seg_cap positions.  rho >= 1 samples everything
 * (up to seg_cap per segment).  Positions come out ascending.  Returns the
 * count, or -1 if out_cap is too small. */
int64_t orc_bernoulli_sample(uint64_t n, double rho, uint64_t seed, uint32_t tag,
                             uint32_t nseg, uint32_t seg_cap,
                             uint32_t *out_pos, uint64_t out_cap)
{
    uint64_t L = (n + nseg - 1) / nseg;
    uint64_t cnt = 0;
    double ln1mrho = rho < 1.0 ? log1p(-rho) : 0.0;
    for (uint32_t t = 0; t < nseg; ++t) {
        uint64_t s = (uint64_t)t * L;
        uint64_t e = s + L < n ? s + L : n;
        if (s >= e) continue;
        uint32_t taken = 0;
        if (rho >= 1.0) {
            for (uint64_t p = s; p < e && taken < seg_cap; ++p, ++taken) {
                if (cnt >= out_cap) return -1;
                out_pos[cnt++] = (uint32_t)p;
            }
            continue;
        }
        int64_t p = (int64_t)s - 1;          /* last position passed */
        uint64_t j = 0;
        while (taken < seg_cap) {
            double u = uniform01(seed, tag, t, j++);
            double q = log(u) / ln1mrho;      /* skip - 1, before flooring */
            /* the next sampled position is p + 1 + floor(q); stop past e-1 */
            if (q >= (double)((int64_t)e - 1 - p)) break;
            p = p + 1 + (int64_t)q;
            if (cnt >= out_cap) return -1;
            out_pos[cnt++] = (uint32_t)p;
            ++taken;
        }
    }
    return (int64_t)cnt;
}

/* ------------------------------------------------------------------------ */
/* Pivot ranks.  FR-selection (§2) takes the sample objects of ranks
 * k|S|/n ± Δ.  With no processor count on one device, Δ is set from the
 * spread of the target's sample rank, a binomial with variance about
 * |S| q (1-q), q = k/n (Chernoff bounds of §2 give the tails):
 *     m_lo = floor(k s / n),  m_hi = ceil(k s / n)
 *     Δ    = ceil(c * sqrt(m_hi (s - m_lo) / s)) + 1,   c = c_num / 4
 *     lo   = m_lo - Δ,        hi = m_hi + Δ            (0-based sample ranks)
 * All integer: ceil(c sqrt(v)) is the least D with 16 s D^2 >= c_num^2 m_hi (s - m_lo).
 * lo < 0 means "no lower pivot" (-inf), hi >= s means "no upper pivot" (+inf). */
static uint64_t ceil_sqrt_u64(uint64_t t)
{
    uint64_t d = (uint64_t)sqrt((double)t);
    while (d * d < t) ++d;
    while (d > 0 && (d - 1) * (d - 1) >= t) --d;
    return d;
}

void orc_pivot_ranks(uint64_t s, uint64_t k, uint64_t n, uint32_t c_num,
                     int64_t *lo, int64_t *hi)
{
    if (s == 0) { *lo = -1; *hi = 0; return; }
    uint64_t m_lo = k * s / n;
    uint64_t m_hi = (k * s + n - 1) / n;
    uint64_t X = (uint64_t)c_num * c_num * m_hi * (s - m_lo);
    uint64_t Y = 16 * s;
    uint64_t t = (X + Y - 1) / Y;
    int64_t delta = (int64_t)ceil_sqrt_u64(t) + 1;
    *lo = (int64_t)m_lo - delta;
    *hi = (int64_t)m_hi + delta;
}

/* ------------------------------------------------------------------------ */
/* Rank of an object: the number of objects that precede it in the unique
 * order (§2).  The k smallest are exactly the objects of rank < k (§4), and a
 * partition of the Algorithm of §2 by pivots l <= r (a = {e < l},
 * b = {l <= e <= r}) has |a| = rank(l) and |b| = rank(r) - rank(l) + 1 within
 * any interval of the order that holds both pivots.  O(n). */
uint64_t orc_rank(const void *keys, int is_f32, uint64_t n, int largest, uint32_t x)
{
    orc_order o = {keys, is_f32, largest};
    uint64_t r = 0;
    for (uint64_t i = 0; i < n; ++i)
        if (i != x && precedes(&o, i, x)) ++r;
    return r;
}

/* Ranks of m objects xs[0..m) among the objects ys[0..q) (positions into
 * keys): out[i] = #{j : ys[j] precedes xs[i]}.  O(m q); for sample-sized sets. */
void orc_rank_among(const void *keys, int is_f32, int largest, const uint32_t *xs, uint64_t m,
                    const uint32_t *ys, uint64_t q, uint64_t *out)
{
    orc_order o = {keys, is_f32, largest};
    for (uint64_t i = 0; i < m; ++i) {
        uint64_t r = 0;
        for (uint64_t j = 0; j < q; ++j)
            if (ys[j] != xs[i] && precedes(&o, ys[j], xs[i])) ++r;
        out[i] = r;
    }
}
