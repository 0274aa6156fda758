/*
 * Random sequential addition of spheres (input generation only).
 *
 * Places spheres one after another, in the order given, at uniformly random
 * positions inside a box, rejecting any position that overlaps a sphere
 * already placed.  A sphere that finds no room after max_attempts tries
 * raises the top of the box by `grow` times its diameter and tries again, so
 * the loop always ends.  Random numbers come from xoshiro256** (Blackman and
 * Vigna) seeded through splitmix64.
 *
 * This is part of the synthetic-input generator: it holds none of the granule
 * method's arithmetic.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    uint64_t s[4];
} rsa_rng;

static uint64_t rsa_splitmix(uint64_t *x)
{
    uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static uint64_t rsa_rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static uint64_t rsa_next(rsa_rng *g)
{
    uint64_t *s = g->s;
    uint64_t out = rsa_rotl(s[1] * 5, 7) * 9;
    uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rsa_rotl(s[3], 45);
    return out;
}

static double rsa_uniform(rsa_rng *g) { return (double)(rsa_next(g) >> 11) * (1.0 / 9007199254740992.0); }

/* pos: 3 x n, structure of arrays.  Returns the final box top (z). */
double rsa_place(int64_t n, const double *rad, const double *lo, const double *hi, double zcap, uint64_t seed,
                 int32_t max_attempts, double grow, double *pos)
{
    rsa_rng g;
    uint64_t sm = seed;
    for (int k = 0; k < 4; ++k) g.s[k] = rsa_splitmix(&sm);
    double rmax = 0.0;
    for (int64_t i = 0; i < n; ++i)
        if (rad[i] > rmax) rmax = rad[i];
    double cs = 2.0 * rmax;
    int64_t nc[3];
    double top[3] = {hi[0], hi[1], zcap};
    for (int a = 0; a < 3; ++a) {
        nc[a] = (int64_t)floor((top[a] - lo[a]) / cs);
        if (nc[a] < 1) nc[a] = 1;
    }
    double csa[3];
    for (int a = 0; a < 3; ++a) csa[a] = (top[a] - lo[a]) / (double)nc[a];
    int64_t ncell = nc[0] * nc[1] * nc[2];
    int64_t *head = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncell);
    int64_t *next = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t c = 0; c < ncell; ++c) head[c] = -1;
    double H = hi[2];
    for (int64_t i = 0; i < n; ++i) {
        double r = rad[i];
        int placed = 0;
        while (!placed) {
            for (int32_t t = 0; t < max_attempts && !placed; ++t) {
                double c[3];
                double span[3] = {hi[0] - lo[0] - 2 * r, hi[1] - lo[1] - 2 * r, H - lo[2] - 2 * r};
                for (int a = 0; a < 3; ++a) c[a] = lo[a] + r + rsa_uniform(&g) * (span[a] > 0 ? span[a] : 0.0);
                int64_t ci[3];
                for (int a = 0; a < 3; ++a) {
                    ci[a] = (int64_t)floor((c[a] - lo[a]) / csa[a]);
                    if (ci[a] < 0) ci[a] = 0;
                    if (ci[a] > nc[a] - 1) ci[a] = nc[a] - 1;
                }
                int clash = 0;
                for (int64_t z = ci[2] - 1; z <= ci[2] + 1 && !clash; ++z)
                    for (int64_t y = ci[1] - 1; y <= ci[1] + 1 && !clash; ++y)
                        for (int64_t x = ci[0] - 1; x <= ci[0] + 1 && !clash; ++x) {
                            if (x < 0 || y < 0 || z < 0 || x >= nc[0] || y >= nc[1] || z >= nc[2]) continue;
                            for (int64_t j = head[(z * nc[1] + y) * nc[0] + x]; j >= 0; j = next[j]) {
                                double d0 = pos[j] - c[0], d1 = pos[n + j] - c[1], d2 = pos[2 * n + j] - c[2];
                                double rr = rad[j] + r;
                                if (d0 * d0 + d1 * d1 + d2 * d2 < rr * rr) {
                                    clash = 1;
                                    break;
                                }
                            }
                        }
                if (!clash) {
                    for (int a = 0; a < 3; ++a) pos[a * n + i] = c[a];
                    int64_t cell = (ci[2] * nc[1] + ci[1]) * nc[0] + ci[0];
                    next[i] = head[cell];
                    head[cell] = i;
                    placed = 1;
                }
            }
            if (!placed) {
                if (H >= zcap) {
                    H = -1.0; /* no room left below zcap */
                    goto done;
                }
                H += grow * 2.0 * r;
                if (H > zcap) H = zcap;
            }
        }
    }
done:
    free(head);
    free(next);
    return H;
}
