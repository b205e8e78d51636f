/*
 * ising_oracle.c — plain CPU oracle (TEST INFRASTRUCTURE ONLY; see ising_oracle.h).
 *
 * Paper: Yang, Chen, Roumpos, Colby, Anderson, "High Performance Monte Carlo
 * Simulation of Ising Model on TPU Clusters" (arXiv 1903.11714).
 *   Sec. 3          Hamiltonian H = -J sum_<ij> s_i s_j - mu sum_i s_i, J = 1, mu = 0,
 *                   periodic (torus) lattice.
 *   Sec. 3.1, eq. 1 checkerboard: with one colour fixed, every site of the other colour
 *                   is offered a Metropolis flip independently; white first, then black.
 *   Sec. 3.2, Alg. 1 nn = sum of the four neighbours; accept where a uniform in [0, 1) is
 *                   below exp(-2 beta nn sigma); flip sigma -> -sigma.
 *   Sec. 4.1        m = (1/N) sum_i sigma_i.
 *   Sec. 4.2        a sweep = one update of all black plus all white sites.
 */
#include "ising_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- Philox4x32-10 (Salmon et al., SC'11, "Parallel random numbers: as easy as 1, 2, 3").
 * One round: the two 32x32 -> 64-bit products M0 * x0 and M1 * x2; the new state is
 * (hi(M1 x2) ^ x1 ^ k0, lo(M1 x2), hi(M0 x0) ^ x3 ^ k1, lo(M0 x0)); the key is bumped by the
 * Weyl constants between rounds, the first round uses the key as given. */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void seed_to_key(uint64_t seed, uint32_t key[2]) {
    key[0] = (uint32_t)(seed & 0xFFFFFFFFu);
    key[1] = (uint32_t)(seed >> 32);
}

/* ---- The site's uniform (Sec. 3.2, Alg. 1 "probs"; Sec. 5.1 random_uniform).
 * All 32 bits are assembled from the eight Philox blocks of the site's group, then used
 * as one unsigned integer. */
uint32_t oracle_uniform(uint64_t seed, uint32_t r, uint32_t c, uint32_t t, int q) {
    uint32_t key[2];
    seed_to_key(seed, key);
    uint32_t j = c >> 1;          /* index among this row's colour-q sites */
    uint32_t g = j >> 5;          /* group of 32 such sites                 */
    uint32_t i = j & 31u;         /* position inside the group              */
    /* bit of each Philox word that belongs to the site: byte (0, 2, 1, 3)[i mod 4], bit i div 4 */
    static const uint32_t byte_of[4] = {0u, 2u, 1u, 3u};
    uint32_t pos = 8u * byte_of[i & 3u] + (i >> 2);
    uint32_t x = 0;
    for (uint32_t m = 0; m < 8; ++m) {
        uint32_t ctr[4] = {g, r, t, 2u * m + (uint32_t)q};
        uint32_t blk[4];
        oracle_philox4x32_10(ctr, key, blk);
        for (uint32_t w = 0; w < 4; ++w) {
            uint32_t k = 4u * m + w;               /* k = 0 is the most significant bit */
            uint32_t bit = (blk[w] >> pos) & 1u;
            x |= bit << (31u - k);
        }
    }
    return x;
}

/* ---- Thresholds.  u = x / 2^32 < p  <=>  x < ceil(p 2^32) for integer x, so the test
 * "uniform < acceptance ratio" of Alg. 1 becomes an exact integer compare. */
void oracle_thresholds(double beta, uint64_t T[2]) {
    for (int k = 0; k < 2; ++k) {
        double s = (k == 0) ? 2.0 : 4.0;
        double p = exp(-2.0 * beta * s);     /* Metropolis ratio for energy change 2 s */
        double y = ceil(ldexp(p, 32));
        if (y > 4294967296.0) y = 4294967296.0;
        if (!(y >= 0.0)) y = 0.0;
        T[k] = (uint64_t)y;
    }
}

/* ---- Hot start. */
int oracle_init_site(uint64_t seed, uint32_t r, uint32_t c) {
    uint32_t key[2];
    seed_to_key(seed, key);
    uint32_t ctr[4] = {c >> 7, r, 0u, 0x80000000u};
    uint32_t blk[4];
    oracle_philox4x32_10(ctr, key, blk);
    uint32_t bit = (blk[(c >> 5) & 3u] >> (c & 31u)) & 1u;
    return bit ? -1 : +1;
}

void oracle_init(int8_t* spins, int64_t L, uint64_t seed) {
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < L; ++r)
        for (int64_t c = 0; c < L; ++c)
            spins[r * L + c] = (int8_t)oracle_init_site(seed, (uint32_t)r, (uint32_t)c);
}

/* ---- Neighbour sum on the torus. */
static int64_t wrap(int64_t a, int64_t L) {
    a %= L;
    return a < 0 ? a + L : a;
}

static int neighbour_sum(const int8_t* s, int64_t L, int64_t r, int64_t c) {
    int64_t up = wrap(r - 1, L), down = wrap(r + 1, L);
    int64_t left = wrap(c - 1, L), right = wrap(c + 1, L);
    return s[up * L + c] + s[down * L + c] + s[r * L + left] + s[r * L + right];
}

void oracle_local_field(const int8_t* spins, int64_t L, int8_t* nn) {
    for (int64_t r = 0; r < L; ++r)
        for (int64_t c = 0; c < L; ++c)
            nn[r * L + c] = (int8_t)neighbour_sum(spins, L, r, c);
}

/* Metropolis decision for one site: s = sigma * nn is half the energy change of a flip. */
static int accept_flip(int sigma, int nn, const uint64_t T[2], uint64_t seed, uint32_t r,
                       uint32_t c, uint32_t t, int q) {
    int s = sigma * nn;
    if (s <= 0) return 1;                  /* min{1, exp(-2 beta s)} = 1 */
    uint64_t thr = (s == 2) ? T[0] : T[1];
    uint64_t x = oracle_uniform(seed, r, c, t, q);
    return x < thr;
}

void oracle_half_sweep(int8_t* spins, int64_t L, const uint64_t T[2], uint64_t seed,
                       uint32_t t, int q) {
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < L; ++r) {
        for (int64_t c = 0; c < L; ++c) {
            if (((r + c) & 1) != q) continue;
            int sigma = spins[r * L + c];
            int nn = neighbour_sum(spins, L, r, c);
            if (accept_flip(sigma, nn, T, seed, (uint32_t)r, (uint32_t)c, t, q))
                spins[r * L + c] = (int8_t)(-sigma);
        }
    }
}

void oracle_observables(const int8_t* spins, int64_t L, int64_t out[2]) {
    int64_t M = 0, E = 0;
    for (int64_t r = 0; r < L; ++r) {
        for (int64_t c = 0; c < L; ++c) {
            int sigma = spins[r * L + c];
            M += sigma;
            /* each bond once: the right and the lower neighbour of every site */
            E -= sigma * (spins[r * L + wrap(c + 1, L)] + spins[wrap(r + 1, L) * L + c]);
        }
    }
    out[0] = M;
    out[1] = E;
}

void oracle_sweep(int8_t* spins, int64_t L, double beta, int64_t n, uint64_t seed,
                  uint64_t offset, int64_t* trace) {
    uint64_t T[2];
    oracle_thresholds(beta, T);
    for (int64_t i = 0; i < n; ++i) {
        uint32_t t = (uint32_t)(offset + (uint64_t)i);
        oracle_half_sweep(spins, L, T, seed, t, 1);   /* white */
        oracle_half_sweep(spins, L, T, seed, t, 0);   /* black */
        if (trace) oracle_observables(spins, L, trace + 2 * i);
    }
}

/* ---- Light-cone crop.  One half-sweep moves information by one lattice step, so after
 * 2 n half-sweeps a site depends only on sites within distance 2 n.  The window is the crop
 * grown by R = 2 n on every side; half-sweep k updates only the part of the window that is
 * still exact afterwards (the crop grown by R - k - 1). */
void oracle_crop(int64_t L, uint64_t seed, double beta, int64_t n, uint64_t offset,
                 int64_t r0, int64_t c0, int64_t h, int64_t w, int8_t* out) {
    int64_t R = 2 * n;
    if (h + 2 * R >= L || w + 2 * R >= L) {
        int8_t* full = (int8_t*)malloc((size_t)(L * L));
        oracle_init(full, L, seed);
        oracle_sweep(full, L, beta, n, seed, offset, NULL);
        for (int64_t a = 0; a < h; ++a)
            for (int64_t b = 0; b < w; ++b)
                out[a * w + b] = full[wrap(r0 + a, L) * L + wrap(c0 + b, L)];
        free(full);
        return;
    }
    int64_t H = h + 2 * R, W = w + 2 * R;
    int8_t* win = (int8_t*)malloc((size_t)(H * W));
    for (int64_t a = 0; a < H; ++a)
        for (int64_t b = 0; b < W; ++b)
            win[a * W + b] = (int8_t)oracle_init_site(seed, (uint32_t)wrap(r0 - R + a, L),
                                                      (uint32_t)wrap(c0 - R + b, L));
    uint64_t T[2];
    oracle_thresholds(beta, T);
    for (int64_t k = 0; k < 2 * n; ++k) {
        uint32_t t = (uint32_t)(offset + (uint64_t)(k / 2));
        int q = (k % 2 == 0) ? 1 : 0;
        int64_t lo = k + 1;
#pragma omp parallel for schedule(static)
        for (int64_t a = lo; a < H - lo; ++a) {
            int64_t r = wrap(r0 - R + a, L);
            for (int64_t b = lo; b < W - lo; ++b) {
                int64_t c = wrap(c0 - R + b, L);
                if (((r + c) & 1) != q) continue;
                int sigma = win[a * W + b];
                int nn = win[(a - 1) * W + b] + win[(a + 1) * W + b] + win[a * W + b - 1] +
                         win[a * W + b + 1];
                if (accept_flip(sigma, nn, T, seed, (uint32_t)r, (uint32_t)c, t, q))
                    win[a * W + b] = (int8_t)(-sigma);
            }
        }
    }
    for (int64_t a = 0; a < h; ++a)
        memcpy(out + a * w, win + (a + R) * W + R, (size_t)w);
    free(win);
}

/* ---- Low-precision acceptance. */
double oracle_round_fmt(double v, int fmt, int toward_zero) {
    if (!(v > 0.0)) return 0.0;                 /* only non-negative values occur here */
    int digits = (fmt == 1) ? 8 : 11;           /* significant bits of bfloat16 / half   */
    int min_exp = (fmt == 1) ? -126 : -14;      /* exponent of the smallest normal       */
    int e;
    frexp(v, &e);                                /* v = m 2^e, m in [0.5, 1)             */
    int lead = e - 1;                            /* v in [2^lead, 2^(lead+1))            */
    if (lead < min_exp) lead = min_exp;          /* subnormal range: fixed quantum        */
    double quantum = ldexp(1.0, lead - (digits - 1));
    double k = v / quantum;                      /* exact: division by a power of two      */
    k = toward_zero ? floor(k) : nearbyint(k);   /* nearbyint: ties to even (default mode) */
    return k * quantum;
}

double oracle_p_fmt(double beta, int s, int fmt) {
    return oracle_round_fmt(exp(-2.0 * beta * (double)s), fmt, 0);
}

double oracle_u_fmt(uint32_t x, int fmt) {
    double r16 = (double)(x >> 16);
    return oracle_round_fmt(ldexp(r16, -16), fmt, 1);
}

static void half_sweep_fmt(int8_t* spins, int64_t L, double beta, int fmt, uint64_t seed, uint32_t t,
                           int q) {
    double p2 = oracle_p_fmt(beta, 2, fmt), p4 = oracle_p_fmt(beta, 4, fmt);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < L; ++r) {
        for (int64_t c = 0; c < L; ++c) {
            if (((r + c) & 1) != q) continue;
            int sigma = spins[r * L + c];
            int s = sigma * neighbour_sum(spins, L, r, c);
            int flip = 1;
            if (s > 0) {
                double u = oracle_u_fmt(oracle_uniform(seed, (uint32_t)r, (uint32_t)c, t, q), fmt);
                flip = u < ((s == 2) ? p2 : p4);
            }
            if (flip) spins[r * L + c] = (int8_t)(-sigma);
        }
    }
}

void oracle_sweep_fmt(int8_t* spins, int64_t L, double beta, int fmt, int64_t n, uint64_t seed,
                      uint64_t offset, int64_t* trace) {
    for (int64_t i = 0; i < n; ++i) {
        uint32_t t = (uint32_t)(offset + (uint64_t)i);
        half_sweep_fmt(spins, L, beta, fmt, seed, t, 1);
        half_sweep_fmt(spins, L, beta, fmt, seed, t, 0);
        if (trace) oracle_observables(spins, L, trace + 2 * i);
    }
}

/* ==== Three dimensions (Sec. 3: the Hamiltonian on a d-dimensional hypercubic lattice; the
 * checkerboard colouring of Fig. 1 extends to any dimension).  Same Metropolis rule, six
 * neighbours, thresholds for s = 2, 4, 6; the random numbers are the 2-D contract's with the
 * row index r = z L + y. */
void oracle3_thresholds(double beta, uint64_t T[3]) {
    for (int k = 0; k < 3; ++k) {
        double p = exp(-2.0 * beta * (2.0 * (k + 1)));   /* s = 2, 4, 6 */
        double y = ceil(ldexp(p, 32));
        if (y > 4294967296.0) y = 4294967296.0;
        if (!(y >= 0.0)) y = 0.0;
        T[k] = (uint64_t)y;
    }
}

void oracle3_init(int8_t* spins, int64_t L, uint64_t seed) {
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < L * L; ++r)           /* r = z L + y */
        for (int64_t x = 0; x < L; ++x)
            spins[r * L + x] = (int8_t)oracle_init_site(seed, (uint32_t)r, (uint32_t)x);
}

static int64_t at3(int64_t L, int64_t z, int64_t y, int64_t x) {
    return (wrap(z, L) * L + wrap(y, L)) * L + wrap(x, L);
}

static int neighbour_sum3(const int8_t* s, int64_t L, int64_t z, int64_t y, int64_t x) {
    return s[at3(L, z - 1, y, x)] + s[at3(L, z + 1, y, x)] + s[at3(L, z, y - 1, x)] +
           s[at3(L, z, y + 1, x)] + s[at3(L, z, y, x - 1)] + s[at3(L, z, y, x + 1)];
}

void oracle3_local_field(const int8_t* spins, int64_t L, int8_t* nn) {
    for (int64_t z = 0; z < L; ++z)
        for (int64_t y = 0; y < L; ++y)
            for (int64_t x = 0; x < L; ++x)
                nn[(z * L + y) * L + x] = (int8_t)neighbour_sum3(spins, L, z, y, x);
}

/* s = sigma nn; s <= 0 always flips, otherwise the uniform of site (z, y, x) is compared with T_s. */
static int accept_flip3(int sigma, int nn, const uint64_t T[3], uint64_t seed, uint32_t r, uint32_t x,
                        uint32_t t, int q) {
    int s = sigma * nn;
    if (s <= 0) return 1;
    uint64_t thr = T[s / 2 - 1];
    return (uint64_t)oracle_uniform(seed, r, x, t, q) < thr;
}

void oracle3_half_sweep(int8_t* spins, int64_t L, const uint64_t T[3], uint64_t seed, uint32_t t, int q) {
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < L * L; ++r) {
        int64_t z = r / L, y = r % L;
        for (int64_t x = 0; x < L; ++x) {
            if (((x + y + z) & 1) != q) continue;
            int sigma = spins[r * L + x];
            int nn = neighbour_sum3(spins, L, z, y, x);
            if (accept_flip3(sigma, nn, T, seed, (uint32_t)r, (uint32_t)x, t, q))
                spins[r * L + x] = (int8_t)(-sigma);
        }
    }
}

void oracle3_observables(const int8_t* spins, int64_t L, int64_t out[2]) {
    int64_t M = 0, E = 0;
    for (int64_t z = 0; z < L; ++z)
        for (int64_t y = 0; y < L; ++y)
            for (int64_t x = 0; x < L; ++x) {
                int sigma = spins[(z * L + y) * L + x];
                M += sigma;
                E -= sigma * (spins[at3(L, z, y, x + 1)] + spins[at3(L, z, y + 1, x)] + spins[at3(L, z + 1, y, x)]);
            }
    out[0] = M;
    out[1] = E;
}

void oracle3_sweep(int8_t* spins, int64_t L, double beta, int64_t n, uint64_t seed, uint64_t offset,
                   int64_t* trace) {
    uint64_t T[3];
    oracle3_thresholds(beta, T);
    for (int64_t i = 0; i < n; ++i) {
        uint32_t t = (uint32_t)(offset + (uint64_t)i);
        oracle3_half_sweep(spins, L, T, seed, t, 1);   /* white */
        oracle3_half_sweep(spins, L, T, seed, t, 0);   /* black */
        if (trace) oracle3_observables(spins, L, trace + 2 * i);
    }
}

/* Light-cone block: after 2 n half-sweeps a site depends only on sites within distance 2 n, so
 * the window is the block grown by R = 2 n on every side, and half-sweep k updates only the part
 * still exact afterwards (the block grown by R - k - 1).  Falls back to the whole lattice when the
 * window would wrap onto itself. */
void oracle3_crop(int64_t L, uint64_t seed, double beta, int64_t n, uint64_t offset, int64_t z0, int64_t y0,
                  int64_t x0, int64_t d, int64_t h, int64_t w, int8_t* out) {
    int64_t R = 2 * n;
    if (d + 2 * R >= L || h + 2 * R >= L || w + 2 * R >= L) {
        int8_t* full = (int8_t*)malloc((size_t)(L * L * L));
        oracle3_init(full, L, seed);
        oracle3_sweep(full, L, beta, n, seed, offset, NULL);
        for (int64_t a = 0; a < d; ++a)
            for (int64_t b = 0; b < h; ++b)
                for (int64_t c = 0; c < w; ++c)
                    out[(a * h + b) * w + c] = full[at3(L, z0 + a, y0 + b, x0 + c)];
        free(full);
        return;
    }
    int64_t D = d + 2 * R, H = h + 2 * R, W = w + 2 * R;
    int8_t* win = (int8_t*)malloc((size_t)(D * H * W));
    for (int64_t a = 0; a < D; ++a)
        for (int64_t b = 0; b < H; ++b)
            for (int64_t c = 0; c < W; ++c)
                win[(a * H + b) * W + c] = (int8_t)oracle_init_site(
                    seed, (uint32_t)(wrap(z0 - R + a, L) * L + wrap(y0 - R + b, L)), (uint32_t)wrap(x0 - R + c, L));
    uint64_t T[3];
    oracle3_thresholds(beta, T);
    for (int64_t k = 0; k < 2 * n; ++k) {
        uint32_t t = (uint32_t)(offset + (uint64_t)(k / 2));
        int q = (k % 2 == 0) ? 1 : 0;
        int64_t lo = k + 1;
#pragma omp parallel for schedule(static)
        for (int64_t a = lo; a < D - lo; ++a) {
            int64_t z = wrap(z0 - R + a, L);
            for (int64_t b = lo; b < H - lo; ++b) {
                int64_t y = wrap(y0 - R + b, L);
                for (int64_t c = lo; c < W - lo; ++c) {
                    int64_t x = wrap(x0 - R + c, L);
                    if (((x + y + z) & 1) != q) continue;
                    int64_t i = (a * H + b) * W + c;
                    int sigma = win[i];
                    int nn = win[i - H * W] + win[i + H * W] + win[i - W] + win[i + W] + win[i - 1] + win[i + 1];
                    if (accept_flip3(sigma, nn, T, seed, (uint32_t)(z * L + y), (uint32_t)x, t, q))
                        win[i] = (int8_t)(-sigma);
                }
            }
        }
    }
    for (int64_t a = 0; a < d; ++a)
        for (int64_t b = 0; b < h; ++b)
            memcpy(out + (a * h + b) * w, win + ((a + R) * H + (b + R)) * W + R, (size_t)w);
    free(win);
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Moments of a traced chain (Sec. 4.1: the magnetisation m = M / N and, for the Binder cumulant,
 * its second and fourth powers; the energy per site e = E / N): out = (<|m|>, <m^2>, <m^4>, <e>, <e^2>)
 * over the n sweeps of trace (M, E pairs), each a plain sum in sweep order divided by n. */
void oracle_moments(const int64_t* trace, int64_t n, int64_t n_sites, double out[5]) {
    double s_abs = 0.0, s_m2 = 0.0, s_m4 = 0.0, s_e = 0.0, s_e2 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double m = (double)trace[2 * i] / (double)n_sites;
        double e = (double)trace[2 * i + 1] / (double)n_sites;
        s_abs += fabs(m);
        s_m2 += m * m;
        s_m4 += (m * m) * (m * m);
        s_e += e;
        s_e2 += e * e;
    }
    out[0] = s_abs / (double)n;
    out[1] = s_m2 / (double)n;
    out[2] = s_m4 / (double)n;
    out[3] = s_e / (double)n;
    out[4] = s_e2 / (double)n;
}
