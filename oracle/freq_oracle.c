/*
 * CPU oracle for the top-k most frequent objects (§7) and the top-k sum
 * aggregation (§8) of Hübschle-Schneider, Sanders, Müller, "Communication
 * Efficient Algorithms for Top-k Selection Problems".
 *
 * TEST INFRASTRUCTURE ONLY (like topk_oracle.c, whose Philox it calls).  It
 * shares no code with the GPU library.  Plain loops over the input: the
 * Bernoulli sample of §7.1 by per-element decisions, exact counting, and the
 * weighted sample of §8 ("Sampling"); the selection of the most frequent
 * objects is done by the Python side with a plain sort.
 *
 * Objects are integers in [0, U).
 */
#include <stdint.h>
#include <string.h>

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]);

/* Bernoulli decision for input position i (§2 "Bernoulli sampling": every
 * element independently with probability rho = T / 2^32): taken iff word
 * i % 4 of Philox4x32-10 at counter (i / 4, 0, tag, 2), key (seed low, seed
 * high), is below T.  T >= 2^32 takes every element, T = 0 none. */
int orc_take(uint64_t seed, uint32_t tag, uint64_t i, uint64_t T)
{
    if (T >= (1ull << 32)) return 1;
    const uint32_t ctr[4] = {(uint32_t)(i >> 2), 0, tag, 2};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    return (uint64_t)w[i & 3] < T;
}

/* Counts of the sampled objects: counts[x] = #{sampled i : keys[i] = x}
 * (§7.1: the sample is counted by object).  *n_sampled = sample size.
 * Returns -1 if a key is outside [0, U). */
int orc_sample_counts(const uint32_t *keys, uint64_t n, uint32_t U, uint64_t seed, uint32_t tag,
                      uint64_t T, uint32_t *counts, uint64_t *n_sampled)
{
    memset(counts, 0, (size_t)U * sizeof(uint32_t));
    uint64_t s = 0;
    for (uint64_t i = 0; i < n; ++i) {
        if (keys[i] >= U) return -1;
        if (orc_take(seed, tag, i, T)) {
            ++counts[keys[i]];
            ++s;
        }
    }
    *n_sampled = s;
    return 0;
}

/* Exact counts: counts[x] = #{i : keys[i] = x} (§7.2's exact counting). */
int orc_exact_counts(const uint32_t *keys, uint64_t n, uint32_t U, uint32_t *counts)
{
    memset(counts, 0, (size_t)U * sizeof(uint32_t));
    for (uint64_t i = 0; i < n; ++i) {
        if (keys[i] >= U) return -1;
        ++counts[keys[i]];
    }
    return 0;
}

/* Aggregated sums of (key, value) pairs: sums[x] = sum of values[i] over
 * keys[i] = x (§8: the input is aggregated by key before it is sampled). */
int orc_sum_by_key(const uint32_t *keys, const uint32_t *values, uint64_t n, uint32_t U,
                   uint64_t *sums)
{
    memset(sums, 0, (size_t)U * sizeof(uint64_t));
    for (uint64_t i = 0; i < n; ++i) {
        if (keys[i] >= U) return -1;
        sums[keys[i]] += values[i];
    }
    return 0;
}

/* Weighted sample of aggregated sums (§8 "Sampling"): with v_avg = m / s
 * (m = the sum of all values, s the desired sample size), object x with sum
 * v_x yields floor(v_x / v_avg) samples directly and one more with
 * probability v_x / v_avg - floor(v_x / v_avg).  In integers: q = floor(v_x s
 * / m), r = v_x s - q m; the extra sample is taken iff word 0 of
 * Philox4x32-10 at counter (x, 0, tag, 3) is below floor(r 2^32 / m).
 * samples[x] receives the count; returns the total, or -1 if m = 0. */
int64_t orc_weighted_sample(const uint64_t *sums, uint32_t U, uint64_t s, uint64_t seed,
                            uint32_t tag, uint32_t *samples)
{
    unsigned __int128 m = 0;
    for (uint32_t x = 0; x < U; ++x) m += sums[x];
    if (m == 0) return -1;
    int64_t total = 0;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (uint32_t x = 0; x < U; ++x) {
        const unsigned __int128 vs = (unsigned __int128)sums[x] * s;
        const unsigned __int128 q = vs / m, r = vs % m;
        const uint64_t thr = (uint64_t)((r << 32) / m);     /* floor(r 2^32 / m) < 2^32 */
        const uint32_t ctr[4] = {x, 0, tag, 3};
        uint32_t w[4];
        orc_philox4x32_10(ctr, key, w);
        const uint64_t c = (uint64_t)q + ((uint64_t)w[0] < thr ? 1u : 0u);
        samples[x] = (uint32_t)c;
        total += (int64_t)c;
    }
    return total;
}
