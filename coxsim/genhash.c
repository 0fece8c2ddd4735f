/*
 * genhash.c -- host generator of synthetic genotype matrices from a counter
 * hash.  Input generation only: no step of the Cox method is computed here.
 *
 * Definition (shared, bit for bit, with the numpy and device versions):
 *   mix(z)        = z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
 *                   z ^= z >> 27; z *= 0x94D049BB133111EB; z ^= z >> 31
 *   splitmix(x)   = mix(x + 0x9E3779B97F4A7C15)           (SplitMix64, Steele,
 *                                                          Lea and Flood 2014)
 *   h(i, j)       = splitmix(((j << 32) | i) ^ splitmix(seed))
 *   G[i, j]       = [low32(h) < t_j] + [high32(h) < t_j]   in {0, 1, 2}
 * where t_j = floor(maf_j * 2^32) is the per-column threshold.  Each of the two
 * alleles is then Bernoulli(maf_j), so G[i, j] ~ Binomial(2, maf_j).
 *
 * Output is column-major: column j starts at byte j * ldx.  fmt 0 writes the
 * count as int8, fmt 1 as its OCP FP8 E4M3 code (0 -> 0x00, 1 -> 0x38,
 * 2 -> 0x40).  Rows n..ldx-1 are left untouched.
 */
#include <stdint.h>

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t splitmix(uint64_t x) { return mix64(x + 0x9E3779B97F4A7C15ULL); }

void coxsim_genotype_host(int8_t *out, int64_t n, int64_t p, int64_t ldx, const int64_t *cols, uint64_t seed,
                          const uint32_t *thresholds, int fmt)
{
    static const int8_t fp8code[3] = {0x00, 0x38, 0x40};
    uint64_t sk = splitmix(seed);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < p; ++c) {
        uint64_t j = cols ? (uint64_t)cols[c] : (uint64_t)c;
        uint32_t t = thresholds[c];
        int8_t *col = out + c * ldx;
        for (int64_t i = 0; i < n; ++i) {
            uint64_t h = splitmix(((j << 32) | (uint64_t)i) ^ sk);
            int g = ((uint32_t)h < t) + ((uint32_t)(h >> 32) < t);
            col[i] = fmt ? fp8code[g] : (int8_t)g;
        }
    }
}

/* Per-column counts of 1s and 2s of an int8 genotype matrix (exact integers). */
void coxsim_genotype_counts_host(const int8_t *G, int64_t n, int64_t p, int64_t ldx, int64_t *c1, int64_t *c2)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < p; ++j) {
        int64_t a = 0, b = 0;
        const int8_t *col = G + j * ldx;
        for (int64_t i = 0; i < n; ++i) {
            a += col[i] == 1;
            b += col[i] == 2;
        }
        c1[j] = a;
        c2[j] = b;
    }
}
