/*
 * Seeded synthetic floe fields: radii, thicknesses and non-overlapping
 * positions per cell.  This is input generation only; it holds none of the
 * method's arithmetic and serves both the HIP path and the FP64 oracle.
 *
 * Random numbers come from one counter-based generator (SplitMix64 finaliser,
 * Steele, Lea & Flood, "Fast splittable pseudorandom number generators",
 * OOPSLA 2014) keyed by (seed, stream, counter), so any cell can be generated
 * on its own and cells can be generated in parallel with identical results.
 *
 * Positions are cell-local unsigned 32-bit fractions of the cell side:
 * x = Lx * xi / 2^32.  Floes are placed largest first by rejection sampling
 * against the doubly periodic images of the floes already placed.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline uint64_t fx_mix64(uint64_t z)
{
    z += 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static inline uint64_t fx_u64(uint64_t seed, uint64_t stream, uint64_t ctr)
{
    return fx_mix64(fx_mix64(seed ^ fx_mix64(stream)) + ctr);
}

static inline double fx_unif(uint64_t seed, uint64_t stream, uint64_t ctr)
{
    /* (0, 1): 53 random bits, offset by half an ulp so log() is safe */
    return ((double)(fx_u64(seed, stream, ctr) >> 11) + 0.5) * 0x1.0p-53;
}

static inline double fx_normal(uint64_t seed, uint64_t stream, uint64_t ctr)
{
    /* Box-Muller, cosine branch, two uniforms per normal */
    double u1 = fx_unif(seed, stream, 2 * ctr);
    double u2 = fx_unif(seed, stream, 2 * ctr + 1);
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

static int fx_cmp_desc(const void* a, const void* b)
{
    float fa = *(const float*)a, fb = *(const float*)b;
    return (fa < fb) - (fa > fb);
}

/* Exposed for tests of the generator itself. */
uint64_t fx_rand_u64(uint64_t seed, uint64_t stream, uint64_t ctr) { return fx_u64(seed, stream, ctr); }

/*
 * Fill floes of cells [0, ncells).  start[c]..start[c+1] are the floe slots of
 * cell c.  Radii: lognormal(median r_med, sigma) clipped to [r_lo, r_hi], then
 * multiplied by r_scale and rounded to float.  Thickness: U[h_lo, h_hi].
 * Returns 0, or -(1 + c) for the first cell c whose placement failed.
 */
int fx_floes(int32_t ncells, const int64_t* start, double Lx, double Ly,
             double r_med, double r_sigma, double r_lo, double r_hi, double r_scale,
             double h_lo, double h_hi, uint64_t seed, int32_t max_tries,
             uint32_t* xi, uint32_t* yi, float* r, float* h)
{
    int failed = 0;
    const double qx = Lx * 0x1.0p-32, qy = Ly * 0x1.0p-32;
#pragma omp parallel for schedule(dynamic, 16)
    for (int32_t c = 0; c < ncells; ++c) {
        if (failed) continue;
        const int64_t s = start[c];
        const int64_t n = start[c + 1] - s;
        if (n <= 0) continue;
        const uint64_t base = (uint64_t)c * 8u;
        float* rc = r + s;
        for (int64_t k = 0; k < n; ++k) {
            double rr = r_med * exp(r_sigma * fx_normal(seed, base + 0, (uint64_t)k));
            if (rr < r_lo) rr = r_lo;
            if (rr > r_hi) rr = r_hi;
            rc[k] = (float)(rr * r_scale);
        }
        qsort(rc, (size_t)n, sizeof(float), fx_cmp_desc);
        for (int64_t k = 0; k < n; ++k)
            h[s + k] = (float)(h_lo + (h_hi - h_lo) * fx_unif(seed, base + 1, (uint64_t)k));
        for (int64_t k = 0; k < n; ++k) {
            int placed = 0;
            for (int32_t t = 0; t < max_tries && !placed; ++t) {
                uint64_t ctr = ((uint64_t)k << 24) | (uint64_t)t;
                uint32_t px = (uint32_t)(fx_u64(seed, base + 2, ctr) >> 32);
                uint32_t py = (uint32_t)(fx_u64(seed, base + 3, ctr) >> 32);
                int ok = 1;
                for (int64_t j = 0; j < k && ok; ++j) {
                    double dx = (double)(int32_t)(px - xi[s + j]) * qx;
                    double dy = (double)(int32_t)(py - yi[s + j]) * qy;
                    double R = (double)rc[k] + (double)rc[j];
                    if (dx * dx + dy * dy <= R * R) ok = 0;
                }
                if (ok) {
                    xi[s + k] = px;
                    yi[s + k] = py;
                    placed = 1;
                }
            }
            if (!placed) {
#pragma omp critical
                { if (!failed) failed = -(1 + c); }
                break;
            }
        }
    }
    return failed;
}
