/*
 * CPU model of the single-instance selection's round policy — TEST
 * INFRASTRUCTURE ONLY, distinct from the oracle.
 *
 * The oracle (oracle/) defines the result: the objects of rank <= k in the
 * unique order of §2.  This model instead mirrors the implementation choices
 * the device makes while it reaches that result, so that a test can compare the
 * device's round trace with an independent CPU run of the same policy:
 *   - the skip sampler of segments (1024 segments, at most 16 draws each);
 *   - the sample of a round's middle part b drawn element by element while b
 *     is formed (word 0 of Philox4x32-10 at counter (x, 0, tag, 1) below
 *     T = s_target 2^32 / expected |b|);
 *   - the retry policy: a miss doubles the pivot spread, a too-wide b halves it;
 *   - the exact fallback once the attempt budget is spent (both pivots become
 *     the object of rank k_cur).
 * None of this decides the selected set (the §2 Algorithm is exact whatever
 * the sample), so parity never rests on this file: it only explains the trace.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    const void *keys;
    int is_f32, largest;
} mdl_order;

static int mdl_less_raw(const mdl_order *o, uint64_t i, uint64_t j)
{
    if (o->is_f32) {
        const float a = ((const float *)o->keys)[i], b = ((const float *)o->keys)[j];
        if (isnan(a)) return 0;
        if (isnan(b)) return 1;
        return a < b;
    }
    return ((const uint32_t *)o->keys)[i] < ((const uint32_t *)o->keys)[j];
}

static int mdl_before(const mdl_order *o, uint64_t i, uint64_t j)
{
    const int lt = o->largest ? mdl_less_raw(o, j, i) : mdl_less_raw(o, i, j);
    if (lt) return 1;
    const int gt = o->largest ? mdl_less_raw(o, i, j) : mdl_less_raw(o, j, i);
    if (gt) return 0;
    return i < j;
}

static int mdl_cmp(const void *pa, const void *pb, void *ctx)
{
    const uint32_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
    if (a == b) return 0;
    return mdl_before((const mdl_order *)ctx, a, b) ? -1 : 1;
}

/* Philox4x32-10 (Salmon et al., SC'11). */
static void mdl_philox(const uint32_t cin[4], uint64_t seed, uint32_t out[4])
{
    uint32_t c0 = cin[0], c1 = cin[1], c2 = cin[2], c3 = cin[3];
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        const uint64_t p0 = 0xD2511F53ull * c0, p1 = 0xCD9E8D57ull * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Skip sampler of the device: segment t of nseg covers [t L, t L + L), draws
 * skips 1 + floor(ln U / ln(1 - rho)), U = (w + 1/2) 2^-32, w word j % 4 of
 * Philox at counter (j / 4, t, tag, 0); at most seg_cap per segment.
 * Returns sequence positions (ascending). */
static int64_t mdl_skip_sample(uint64_t n, double rho, uint64_t seed, uint32_t tag,
                               uint32_t nseg, uint32_t seg_cap, uint32_t *pos, uint64_t cap)
{
    const uint64_t L = (n + nseg - 1) / nseg;
    const double l1 = rho < 1.0 ? log1p(-rho) : 0.0;
    uint64_t cnt = 0;
    for (uint32_t t = 0; t < nseg; ++t) {
        const uint64_t s = (uint64_t)t * L, e = s + L < n ? s + L : n;
        if (s >= e) continue;
        uint32_t taken = 0;
        if (rho >= 1.0) {
            for (uint64_t p = s; p < e && taken < seg_cap; ++p, ++taken) {
                if (cnt >= cap) return -1;
                pos[cnt++] = (uint32_t)p;
            }
            continue;
        }
        int64_t p = (int64_t)s - 1;
        uint32_t w[4];
        for (uint64_t j = 0; taken < seg_cap; ++j) {
            if ((j & 3) == 0) {
                const uint32_t c[4] = {(uint32_t)(j >> 2), t, tag, 0};
                mdl_philox(c, seed, w);
            }
            const double u = ((double)w[j & 3] + 0.5) * (1.0 / 4294967296.0);
            const double q = log(u) / l1;
            if (q >= (double)((int64_t)e - 1 - p)) break;
            p = p + 1 + (int64_t)q;
            if (cnt >= cap) return -1;
            pos[cnt++] = (uint32_t)p;
            ++taken;
        }
    }
    return (int64_t)cnt;
}

/* Integer pivot ranks of the device (R4 reading of §2's FR-selection). */
static void mdl_ranks(uint64_t s, uint64_t k, uint64_t n, uint32_t c_num, int64_t *lo, int64_t *hi)
{
    if (s == 0) { *lo = -1; *hi = 0; return; }
    const uint64_t m_lo = k * s / n, m_hi = (k * s + n - 1) / n;
    const uint64_t X = (uint64_t)c_num * c_num * m_hi * (s - m_lo), Y = 16 * s;
    const uint64_t t = (X + Y - 1) / Y;
    uint64_t d = (uint64_t)sqrt((double)t);
    while (d * d < t) ++d;
    while (d > 0 && (d - 1) * (d - 1) >= t) --d;
    *lo = (int64_t)m_lo - (int64_t)(d + 1);
    *hi = (int64_t)m_hi + (int64_t)(d + 1);
}

int mdl_hash_taken(uint64_t seed, uint32_t tag, uint32_t x, uint64_t T)
{
    const uint32_t c[4] = {x, 0, tag, 1};
    uint32_t w[4];
    mdl_philox(c, seed, w);
    return (uint64_t)w[0] < T;
}

uint64_t mdl_band_threshold(uint64_t n_cur, uint64_t s, int64_t lo, int64_t hi, uint64_t s_target)
{
    uint64_t nb = n_cur;
    if (s > 0) {
        const int64_t bot = lo >= 0 ? lo : 0, top = hi < (int64_t)s ? hi + 1 : (int64_t)s;
        nb = n_cur * (uint64_t)(top - bot) / s;
    }
    if (nb == 0) nb = 1;
    return (s_target << 32) / nb;
}

typedef struct {
    uint32_t n_cur, k_cur, s, c_num;
    int64_t lo, hi;
    uint32_t l_idx, r_idx, has_l, has_r;
    uint32_t na, nb, ok, tag;
} mdl_round;

typedef struct {
    uint32_t s_target, c_num, nseg, seg_cap, t_fin, r_max;
    uint64_t band_cap, seed;
    uint32_t s_max, pad;
} mdl_params;

#define MDL_ROUND_EXACT (-2)

/* Run the policy.  Returns 0 (out_idx[k] holds the selection in the order the
 * rounds write it, *kth_idx the object of rank k), or < 0 on an internal
 * error.  recs receives at most max_recs rounds; *nrecs counts them all. */
int mdl_replay(const void *keys, int is_f32, uint64_t n, uint64_t k, int largest,
               const mdl_params *prm, uint32_t *out_idx, uint32_t *kth_idx,
               mdl_round *recs, uint32_t max_recs, uint32_t *nrecs)
{
    if (n == 0 || k == 0 || k > n || n > 0xFFFFFFFFull) return -1;
    mdl_order o = {keys, is_f32, largest};
    const uint32_t smax = prm->nseg * prm->seg_cap;
    uint32_t *cur = malloc(n * sizeof(uint32_t)), *nxt = malloc(n * sizeof(uint32_t));
    uint32_t *spos = malloc((smax + 1) * sizeof(uint32_t)), *samp = malloc((smax + 1) * sizeof(uint32_t));
    uint32_t *hsamp = malloc(((uint64_t)prm->s_max + 1) * sizeof(uint32_t));
    if (!cur || !nxt || !spos || !samp || !hsamp) return -2;
    for (uint64_t i = 0; i < n; ++i) cur[i] = (uint32_t)i;
    uint64_t n_cur = n, k_cur = k, cursor = 0;
    uint32_t c_num = prm->c_num, tag = 0, nr = 0;
    int64_t hcount = -1;
    int status = 0;
    for (;;) {
        if (n_cur <= prm->t_fin) {
            memcpy(nxt, cur, n_cur * sizeof(uint32_t));
            qsort_r(nxt, n_cur, sizeof(uint32_t), mdl_cmp, &o);
            const uint32_t tau = nxt[k_cur - 1];
            uint64_t w = 0;
            for (uint64_t i = 0; i < n_cur; ++i)
                if (cur[i] == tau || mdl_before(&o, cur[i], tau)) out_idx[cursor + w++] = cur[i];
            *kth_idx = tau;
            if (w != k_cur) status = -3;
            break;
        }
        int64_t s = 0, lo, hi;
        int has_l, has_r;
        uint32_t l, r;
        const int exact = tag >= prm->r_max;
        if (exact) {
            /* both pivots: the object of rank k_cur of the subproblem */
            memcpy(nxt, cur, n_cur * sizeof(uint32_t));
            qsort_r(nxt, n_cur, sizeof(uint32_t), mdl_cmp, &o);
            l = r = nxt[k_cur - 1];
            lo = hi = MDL_ROUND_EXACT;
            has_l = has_r = 1;
        } else {
            if (hcount >= 0) {
                s = hcount;
                for (int64_t i = 0; i < s; ++i) samp[i] = hsamp[i];
            } else {
                s = mdl_skip_sample(n_cur, (double)prm->s_target / (double)n_cur, prm->seed, tag,
                                    prm->nseg, prm->seg_cap, spos, smax);
                if (s < 0) { status = -4; break; }
                for (int64_t i = 0; i < s; ++i) samp[i] = cur[spos[i]];
            }
            qsort_r(samp, (size_t)s, sizeof(uint32_t), mdl_cmp, &o);
            mdl_ranks((uint64_t)s, k_cur, n_cur, c_num, &lo, &hi);
            has_l = lo >= 0;
            has_r = hi < s;
            l = has_l ? samp[lo] : 0;
            r = has_r ? samp[hi] : 0;
        }
        hcount = -1;
        uint64_t na = 0, nb = 0, hs = 0;
        const uint64_t T = exact ? 0 : mdl_band_threshold(n_cur, (uint64_t)s, lo, hi, prm->s_target);
        for (uint64_t i = 0; i < n_cur; ++i) {
            const uint32_t e = cur[i];
            if (has_l && e != l && mdl_before(&o, e, l)) {
                if (cursor + na < k) out_idx[cursor + na] = e;
                ++na;
            } else if (has_r && e != r && mdl_before(&o, r, e)) {
                /* c: dropped */
            } else {
                if (nb < prm->band_cap) nxt[nb] = e;
                ++nb;
                if (mdl_hash_taken(prm->seed, tag + 1, e, T)) {
                    if (hs < prm->s_max) hsamp[hs] = e;
                    ++hs;
                }
            }
        }
        const int miss = na >= k_cur || na + nb < k_cur;
        const int wide = nb > prm->band_cap || nb == n_cur;
        const int ok = !miss && !wide;
        if (recs && nr < max_recs) {
            mdl_round *R = &recs[nr];
            R->n_cur = (uint32_t)n_cur; R->k_cur = (uint32_t)k_cur; R->s = (uint32_t)s;
            R->c_num = c_num; R->lo = lo; R->hi = hi;
            R->l_idx = has_l ? l : 0; R->r_idx = has_r ? r : 0;
            R->has_l = has_l; R->has_r = has_r;
            R->na = (uint32_t)na; R->nb = (uint32_t)nb; R->ok = ok; R->tag = tag;
        }
        ++nr;
        ++tag;
        if (miss) {
            if (exact) { status = -5; break; }
            c_num = c_num * 2 > 4096 ? 4096 : c_num * 2;
            continue;
        }
        if (wide) {
            if (exact) { status = -5; break; }
            c_num /= 2;
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
