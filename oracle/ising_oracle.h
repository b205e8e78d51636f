/*
 * ising_oracle.h — plain CPU oracle for the checkerboard Metropolis sweep of the
 * periodic 2D Ising model (Yang et al., "High Performance Monte Carlo Simulation
 * of Ising Model on TPU Clusters", arXiv 1903.11714).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke entry point and the
 * benchmark's CPU-baseline leg may load or call this code.  It shares nothing with
 * the HIP path: its own Philox, thresholds, initial state, sweep and observables.
 *
 * Everything is written for clarity, not speed: one site at a time, the site's
 * 32-bit uniform assembled from all eight Philox blocks that feed it, doubles for
 * the thresholds.  Parallel loops (OpenMP over rows of one half-sweep) are the only
 * concession; they cannot change results because every site of one colour reads
 * only sites of the other colour and the random numbers are counter based.
 *
 * Conventions (shared by contract with the HIP path, implemented separately):
 *   lattice    int8, row-major L x L, values +1 / -1, periodic in both axes (Sec. 3).
 *   colour     q(r, c) = (r + c) & 1; q = 0 "black", q = 1 "white" (Sec. 3.2, mask M
 *              has M[0][0] = 1 for black).
 *   sweep t    white half-sweep (q = 1) then black (q = 0) (Sec. 3.1, the two
 *              alternating sub-routines, white updated first).
 *   uniform    x(r, c, t) is a 32-bit unsigned integer, u = x / 2^32 in [0, 1).
 *              With j = c >> 1 (index of the site among its row's colour-q sites),
 *              g = j >> 5, i = j & 31 and p(i) = 8 * b(i & 3) + (i >> 2), b = (0, 2, 1, 3):
 *              bit (31 - k) of x, k = 0..31, is bit p(i) of word (k & 3) of
 *              Philox4x32-10(key = (seed mod 2^32, seed >> 32),
 *                            counter = (g, r, t, 2 * (k >> 2) + q)).
 *   threshold  T_s = ceil(2^32 * exp(-2 * beta * s)) for s in {2, 4}; a site with
 *              s = sigma * nn <= 0 always flips, otherwise flips iff x < T_s
 *              (Sec. 3.2, Algorithm 1: flip where the uniform is below the
 *              acceptance ratio; beta restored in the exponent, Sec. 3).
 *   init       hot start: sigma0(r, c) = -1 iff bit (c & 31) of word ((c >> 5) & 3)
 *              of Philox4x32-10(key, counter = (c >> 7, r, 0, 0x80000000)) is set.
 */
#ifndef ISING_ORACLE_H
#define ISING_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): out = bijection of ctr under key. */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* The site's 32-bit uniform for half-sweep (t, q). */
uint32_t oracle_uniform(uint64_t seed, uint32_t r, uint32_t c, uint32_t t, int q);

/* Acceptance thresholds: T[0] = T_2, T[1] = T_4, each in [0, 2^32]. */
void oracle_thresholds(double beta, uint64_t T[2]);

/* Hot-start spin of one site, and of a whole lattice. */
int oracle_init_site(uint64_t seed, uint32_t r, uint32_t c);
void oracle_init(int8_t* spins, int64_t L, uint64_t seed);

/* Sum of the four periodic nearest neighbours of every site (Sec. 3.2, nn(sigma)). */
void oracle_local_field(const int8_t* spins, int64_t L, int8_t* nn);

/* One colour update in place: every site of colour q is offered a flip. */
void oracle_half_sweep(int8_t* spins, int64_t L, const uint64_t T[2], uint64_t seed,
                       uint32_t t, int q);

/* n sweeps, sweep indices t = offset .. offset + n - 1.  If trace != NULL it receives
 * (M, E) after every sweep, trace[2 * i] = M, trace[2 * i + 1] = E. */
void oracle_sweep(int8_t* spins, int64_t L, double beta, int64_t n, uint64_t seed,
                  uint64_t offset, int64_t* trace);

/* out[0] = M = sum of spins, out[1] = E = -sum over the 2 L^2 bonds of sigma_i sigma_j. */
void oracle_observables(const int8_t* spins, int64_t L, int64_t out[2]);

/* The h x w crop with top-left corner (r0, c0) (taken mod L) of the lattice obtained
 * from the hot start of `seed` after n sweeps from offset, computed on a window that
 * holds every site the crop can depend on (light cone of 2 n half-sweeps). */
void oracle_crop(int64_t L, uint64_t seed, double beta, int64_t n, uint64_t offset,
                 int64_t r0, int64_t c0, int64_t h, int64_t w, int8_t* out);

/* ---- Low-precision acceptance (the paper's bfloat16 experiment, Sec. 4.1).
 * fmt 1 = bfloat16 (8 significant bits, float32 exponent range), fmt 2 = IEEE half (11
 * significant bits, smallest normal 2^-14, subnormals down to 2^-24).
 *   p_fmt(s) = exp(-2 beta s) rounded to nearest-even in fmt (one rounding from double);
 *   u_fmt    = (top 16 bits of the site's uniform x) / 2^16, rounded toward zero in fmt;
 *   a site with s > 0 flips iff u_fmt < p_fmt (compared as real numbers).
 * The random numbers are the exact chain's, so both chains see identical draws. */
double oracle_round_fmt(double v, int fmt, int toward_zero);
double oracle_p_fmt(double beta, int s, int fmt);
double oracle_u_fmt(uint32_t x, int fmt);
void oracle_sweep_fmt(int8_t* spins, int64_t L, double beta, int fmt, int64_t n, uint64_t seed,
                      uint64_t offset, int64_t* trace);

/* ---- Three dimensions (the d-dimensional hypercubic lattice of Sec. 3; the checkerboard
 * colouring extends to any dimension, Fig. 1).  An L x L x L torus, L even, stored z-major:
 * site (z, y, x) at index (z L + y) L + x.  Colour q = (x + y + z) mod 2, white (q = 1) first.
 * nn = sum of the six neighbours, s = sigma nn in {-6, ..., 6}; a site flips iff s <= 0 or its
 * uniform is below T_s = ceil(2^32 exp(-2 beta s)), s in {2, 4, 6}.  Random numbers: the 2-D
 * contract with row index r = z L + y (oracle_uniform(seed, z L + y, x, t, q)), hot start
 * oracle_init_site(seed, z L + y, x). */
void oracle3_thresholds(double beta, uint64_t T[3]);
void oracle3_init(int8_t* spins, int64_t L, uint64_t seed);
void oracle3_local_field(const int8_t* spins, int64_t L, int8_t* nn);
void oracle3_half_sweep(int8_t* spins, int64_t L, const uint64_t T[3], uint64_t seed, uint32_t t, int q);
void oracle3_sweep(int8_t* spins, int64_t L, double beta, int64_t n, uint64_t seed, uint64_t offset,
                   int64_t* trace);
/* out[0] = M, out[1] = E = -sum over the 3 L^3 bonds (each site's +x, +y, +z neighbour). */
void oracle3_observables(const int8_t* spins, int64_t L, int64_t out[2]);
/* The d x h x w block with corner (z0, y0, x0) (mod L) after n sweeps from the hot start,
 * computed on the light-cone window (the block grown by 2 n on every side). */
void oracle3_crop(int64_t L, uint64_t seed, double beta, int64_t n, uint64_t offset, int64_t z0, int64_t y0,
                  int64_t x0, int64_t d, int64_t h, int64_t w, int8_t* out);

/* Number of OpenMP threads the oracle's parallel loops use (1 without OpenMP). */
int oracle_num_threads(void);

/* Threads of the OpenMP loops from now on (n > 0). */
void oracle_set_num_threads(int n);

/* (<|m|>, <m^2>, <m^4>, <e>, <e^2>) of a traced chain, m = M / n_sites, e = E / n_sites, plain FP64
 * sums in sweep order (Sec. 4.1). */
void oracle_moments(const int64_t* trace, int64_t n, int64_t n_sites, double out[5]);

#ifdef __cplusplus
}
#endif

#endif
