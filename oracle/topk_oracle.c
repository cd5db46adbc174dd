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
 *   - an O(n) checker of a claimed result      (invariants of the selection problem)
 *   - Philox4x32-10                             (Salmon et al., SC'11, published definition)
 *   - Bernoulli sampling with geometric skips  (§2, "Bernoulli sampling")
 *   - pivot ranks around k|S|/n ± Δ            (§2, distributed FR-selection; §4.1 proof)
 *   - a replay of the recursive three-way partition selection
 *                                               (§2, Algorithm "communication efficient
 *                                                selection"; §4.1, Theorem "selectFR")
 *
 * All integer results are exact.  The only floating point is inside the skip
 * computation of the sampler (fp64 log), which decides sample positions only.
 */
#define _GNU_SOURCE
#include <math.h>
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
/* Bernoulli sample by per-element decisions (§2, "Bernoulli sampling": every
 * object is taken independently with probability rho).  Used for the sample of
 * a subproblem that is being produced element by element: object x (input
 * position) is taken iff word 0 of Philox4x32-10 at counter (x, 0, tag, 1)
 * with key = seed is below T = floor(rho 2^32) (T >= 2^32: every object). */
int orc_hash_taken(uint64_t seed, uint32_t tag, uint32_t x, uint64_t T)
{
    uint32_t ctr[4] = {x, 0, tag, 1};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return (uint64_t)out[0] < T;
}

/* Rate of that sample for the middle part b of a round: the pivots cover the
 * sample ranks [bot, top) with bot = lo (0 without a lower pivot) and
 * top = hi + 1 (s without an upper pivot), so b is expected to hold about
 * n_cur (top - bot) / s elements; rho = s_target / that, as T = rho 2^32. */
uint64_t orc_band_threshold(uint64_t n_cur, uint64_t s, int64_t lo, int64_t hi,
                            uint64_t s_target)
{
    uint64_t nb_est = n_cur;
    if (s > 0) {
        int64_t bot = lo >= 0 ? lo : 0;
        int64_t top = hi < (int64_t)s ? hi + 1 : (int64_t)s;
        nb_est = n_cur * (uint64_t)(top - bot) / s;
    }
    if (nb_est == 0) nb_est = 1;
    uint64_t T = (s_target << 32) / nb_est;
    return T;
}

/* ------------------------------------------------------------------------ */
/* Replay of the recursive selection (§2, Algorithm "communication efficient
 * selection", with the sampling of §4.1), step by step, on one address space.
 *
 * Round:  sample the current subproblem at rate s_target / n_cur; sort the
 * sample; pick pivots l = S[lo], r = S[hi]; partition the current sequence
 * into a = {e < l}, b = {l <= e <= r}, c = {e > r}; n_a = |a|, n_b = |b|.
 * Elements of a are written (in sequence order) to out_idx after the
 * `cursor` elements already fixed; b (in sequence order) becomes the next
 * subproblem; k_cur -= n_a.  A round is repeated on the same subproblem with
 * a fresh random stream when its pivots do not bracket rank k_cur (n_a >=
 * k_cur or n_a + n_b < k_cur; this replaces the recursion into a or c, with
 * the same result) -- then with c doubled -- or when b is too wide (more
 * than band_cap elements, or n_b = n_cur: no progress) -- then with c halved.
 * After a recursion into b, c returns to its initial value.  Once
 * n_cur <= t_fin the subproblem is solved
 * directly: tau = its element of rank k_cur; every element <= tau (in sequence
 * order) is written after the cursor.  More than r_max rounds: status 1.
 *
 * Samples.  The first attempt on the input, and every repeated attempt, uses
 * the skip sampler over the current sequence with stream (seed, tag,
 * segment).  After a recursion into b, the next attempt's sample is drawn
 * while b is formed: each element of b is taken by the per-element rule
 * (orc_hash_taken) with stream tag + 1 and the rate of orc_band_threshold; if
 * that sample exceeds s_max elements it is discarded and the skip sampler is
 * used instead.  The sample is a set: the pivots depend only on its members.
 * Each round is recorded in recs[]. */
typedef struct {
    uint32_t n_cur, k_cur;       /* subproblem before the round               */
    uint32_t s;                  /* sample size                                */
    uint32_t c_num;              /* pivot spread factor used (c = c_num / 4)   */
    int64_t lo, hi;              /* pivot sample ranks                         */
    uint32_t l_idx, r_idx;       /* pivot objects (input positions); 0 if none */
    uint32_t has_l, has_r;
    uint32_t na, nb;             /* partition counts                           */
    uint32_t ok;                 /* 1: recursed into b; 0: round repeated      */
    uint32_t tag;                /* random stream of this round                */
} orc_round;

typedef struct {
    uint32_t s_target;           /* expected sample size                       */
    uint32_t c_num;              /* initial spread factor numerator (c = /4)   */
    uint32_t nseg, seg_cap;      /* skip sampler segmentation                  */
    uint32_t t_fin;              /* solve directly at or below this size       */
    uint32_t r_max;              /* attempt budget                             */
    uint64_t band_cap;           /* capacity for b                             */
    uint64_t seed;
    uint32_t s_max;              /* largest usable sample                      */
    uint32_t pad;
} orc_params;

int orc_replay(const void *keys, int is_f32, uint64_t n, uint64_t k, int largest,
               const orc_params *prm, uint32_t *out_idx, uint32_t *kth_idx,
               orc_round *recs, uint32_t *nrecs)
{
    if (n == 0 || k == 0 || k > n || n > 0xFFFFFFFFull) return -1;
    orc_order o = {keys, is_f32, largest};
    uint32_t *cur = (uint32_t *)malloc(n * sizeof(uint32_t));
    uint32_t *nxt = (uint32_t *)malloc(n * sizeof(uint32_t));
    uint32_t smax = prm->nseg * prm->seg_cap;
    uint32_t *spos = (uint32_t *)malloc((smax + 1) * sizeof(uint32_t));
    uint32_t *samp = (uint32_t *)malloc((smax + 1) * sizeof(uint32_t));
    if (!cur || !nxt || !spos || !samp) return -2;
    for (uint64_t i = 0; i < n; ++i) cur[i] = (uint32_t)i;
    uint64_t n_cur = n, k_cur = k, cursor = 0;
    uint32_t c_num = prm->c_num, tag = 0, nr = 0;
    uint32_t *hsamp = (uint32_t *)malloc(((uint64_t)prm->s_max + 1) * sizeof(uint32_t));
    int64_t hcount = -1;         /* size of the per-element sample of cur; -1: none */
    int status = 0;
    if (!hsamp) return -2;
    for (;;) {
        if (n_cur <= prm->t_fin) {
            /* base case: sort the small subproblem, tau = rank k_cur */
            memcpy(nxt, cur, n_cur * sizeof(uint32_t));
            qsort_r(nxt, n_cur, sizeof(uint32_t), cmp_idx, &o);
            uint32_t tau = nxt[k_cur - 1];
            uint64_t w = 0;
            for (uint64_t i = 0; i < n_cur; ++i)
                if (cur[i] == tau || precedes(&o, cur[i], tau))
                    out_idx[cursor + w++] = cur[i];
            *kth_idx = tau;
            if (w != k_cur) status = -3;
            break;
        }
        if (tag >= prm->r_max) { status = 1; break; }
        int64_t s;
        if (hcount >= 0) {
            s = hcount;
            for (int64_t i = 0; i < s; ++i) samp[i] = hsamp[i];
        } else {
            double rho = (double)prm->s_target / (double)n_cur;
            s = orc_bernoulli_sample(n_cur, rho, prm->seed, tag, prm->nseg,
                                     prm->seg_cap, spos, smax);
            if (s < 0) { status = -4; break; }
            for (int64_t i = 0; i < s; ++i) samp[i] = cur[spos[i]];
        }
        hcount = -1;
        qsort_r(samp, (size_t)s, sizeof(uint32_t), cmp_idx, &o);
        int64_t lo, hi;
        orc_pivot_ranks((uint64_t)s, k_cur, n_cur, c_num, &lo, &hi);
        int has_l = lo >= 0, has_r = hi < s;
        uint32_t l = has_l ? samp[lo] : 0, r = has_r ? samp[hi] : 0;
        uint64_t na = 0, nb = 0, hs = 0;
        uint64_t T = orc_band_threshold(n_cur, (uint64_t)s, lo, hi, prm->s_target);
        for (uint64_t i = 0; i < n_cur; ++i) {
            uint32_t e = cur[i];
            if (has_l && precedes(&o, e, l)) {
                if (cursor + na < k) out_idx[cursor + na] = e;
                ++na;
            } else if (has_r && precedes(&o, r, e)) {
                /* part c: dropped */
            } else {
                if (nb < prm->band_cap) nxt[nb] = e;
                ++nb;
                if (orc_hash_taken(prm->seed, tag + 1, e, T)) {
                    if (hs < prm->s_max) hsamp[hs] = e;
                    ++hs;
                }
            }
        }
        int miss = na >= k_cur || na + nb < k_cur;
        int wide = nb > prm->band_cap || nb == n_cur;
        int ok = !miss && !wide;
        if (recs) {
            orc_round *R = &recs[nr];
            R->n_cur = (uint32_t)n_cur; R->k_cur = (uint32_t)k_cur; R->s = (uint32_t)s;
            R->c_num = c_num; R->lo = lo; R->hi = hi;
            R->l_idx = l; R->r_idx = r; R->has_l = has_l; R->has_r = has_r;
            R->na = (uint32_t)na; R->nb = (uint32_t)nb; R->ok = ok; R->tag = tag;
        }
        ++nr;
        ++tag;
        if (miss) {
            c_num = c_num * 2 > 4096 ? 4096 : c_num * 2;
            continue;
        }
        if (wide) {
            c_num = c_num / 2;
            continue;
        }
        cursor += na;
        k_cur -= na;
        n_cur = nb;
        uint32_t *t = cur; cur = nxt; nxt = t;
        c_num = prm->c_num;
        hcount = hs <= prm->s_max ? (int64_t)hs : -1;
    }
    if (nrecs) *nrecs = nr;
    free(cur); free(nxt); free(spos); free(samp); free(hsamp);
    return status;
}
