// ising.hip — checkerboard Metropolis sweep of the periodic 2D Ising model on gfx950.
//
// Paper: Yang, Chen, Roumpos, Colby, Anderson, "High Performance Monte Carlo Simulation of
// Ising Model on TPU Clusters" (arXiv 1903.11714).  The update rule is Sec. 3.1 (eq. 1: with
// one colour fixed, all sites of the other colour are independent; white first, then black)
// and Sec. 3.2 Algorithm 1 (neighbour sum, accept where the uniform is below the Metropolis
// ratio, flip).  The paper computes the neighbour sum with matrix products on the TPU's MXU;
// here it is a bit-parallel stencil on the vector ALU, because the update is a memory-bound
// 4-point integer stencil and not a dense contraction.
//
// int8 half-sweep kernel, one launch per colour:
//   * a lane owns one 64-column segment ("group": its 32 same-colour sites share Philox
//     blocks) of a strip of R consecutive rows and streams down the strip, so every row is
//     read from HBM once per half-sweep (plus one halo row above and below the strip);
//   * each row's 64 bytes are reduced to two 32-bit words of sign bits, one per colour, with
//     one byte-permute per pair of dwords; the neighbour count, the acceptance decision and
//     the observables all work on those bit words, 32 sites per instruction;
//   * the site's 32-bit uniform is compared with its threshold one bit plane at a time, most
//     significant first, four planes per Philox block, stopping as soon as no site of the
//     wave is still tied with its threshold (the result is the exact x < T);
//   * flips go back into the bytes with a sign-extending byte permute and one xor.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <atomic>
#include <queue>
#include <string>
#include <tuple>
#include <vector>

#include "ising.h"
#include "philox.hpp"
#include "host.hpp"
#include "rows.hpp"

namespace ising {


// One row of the half-sweep for colour Q.  O = column parity of the colour-Q sites of this row.
// bprev: row r-1 sites at parity O (vertical neighbours), bcur: row r sites at parity 1-O
// (horizontal neighbours).  Returns row r+1's sites at parity O (the next row's bcur).
// The Metropolis decision for the 32 colour-Q sites of one group of one row, all in bit words
// (site order): a = the sites, up/down = the vertical neighbours, side = the horizontal
// neighbour with the same site index, hs = the other horizontal neighbour.  Returns the flip
// mask; with OBS it also counts the anti-aligned bonds of these sites after the update and
// the -1 spins among these sites (after) plus `others` (the other colour of the row).
template <int Q, bool OBS>
// `valid` marks the sites that exist (all 32 except in a row of only 16 same-colour sites).
__device__ __forceinline__ uint32_t decide(uint32_t a, uint32_t up, uint32_t down, uint32_t side, uint32_t hs,
                                           uint32_t others, const Thresholds& th, uint32_t g, uint32_t r,
                                           uint32_t t, uint32_t key0, uint32_t key1, Counts& cnt,
                                           uint32_t valid = 0xFFFFFFFFu) {
    const uint32_t x1 = a ^ up, x2 = a ^ down, x3 = a ^ side, x4 = a ^ hs;  // anti-aligned
    const uint32_t o12 = x1 | x2, o34 = x3 | x4;
    const uint32_t ge2 = ((x1 & x2) | (x3 & x4) | (o12 & o34)) & valid;  // >= 2 anti-aligned: s <= 0
    const uint32_t any = o12 | o34;
    const uint32_t sel2 = any & ~ge2 & valid;                              // exactly one: s = 2
    const uint32_t sel4 = ~any & valid;                                    // none: s = 4
    const uint32_t F = ge2 | accept_mask(sel2, sel4, th, g, r, t, (uint32_t)Q, key0, key1);
    if (OBS) {
        cnt.anti += __builtin_popcount((x1 ^ F) & valid) + __builtin_popcount((x2 ^ F) & valid) +
                    __builtin_popcount((x3 ^ F) & valid) + __builtin_popcount((x4 ^ F) & valid);
        cnt.neg += __builtin_popcount((a ^ F) & valid) + __builtin_popcount(others & valid);
    }
    return F;
}

// One row of the int8 half-sweep for colour Q.  O = column parity of the colour-Q sites of this
// row.  bprev: row r-1 sites at parity O (vertical neighbours), bcur: row r sites at parity 1-O
// (horizontal neighbours).  Returns row r+1's sites at parity O (the next row's bcur).
// `half`: this group is a half group (16 sites per colour, the last group of a row whose length is an
// odd multiple of 32).
template <int Q, int O, bool OBS>
__device__ __forceinline__ uint32_t sweep_row(Row& cur, const Row& nxt, uint32_t bprev, uint32_t bcur,
                                              uint32_t halo, const Thresholds& th, uint32_t g,
                                              uint32_t r, uint32_t t, uint32_t key0, uint32_t key1,
                                              Counts& cnt, bool half = false) {
    const uint32_t bnext = site_bits<O>(nxt);
    const uint32_t a = site_bits<O>(cur);
    // horizontal neighbour that lies in the adjacent group: byte 0 of the right halo dword
    // (O = 1) or byte 3 of the left halo dword (O = 0); bit 1 of a byte is its sign
    const uint32_t hs = O == 1 ? (half ? shift_next_half(bcur, (halo >> 1) & 1u) : shift_next(bcur, (halo >> 1) & 1u))
                               : shift_prev(bcur, (halo >> 25) & 1u);
    const uint32_t F = decide<Q, OBS>(a, bprev, bnext, bcur, hs, bcur, th, g, r, t, key0, key1, cnt,
                                      half ? kHalfSites : 0xFFFFFFFFu);
    apply_flips<O>(cur, F);
    return bnext;
}

struct SweepArgs {
    int8_t* spins;
    uint32_t L, groups, rows, n_lanes;  // rows = rows per lane (even, divides L)
    uint32_t t, key0, key1;
    Thresholds th;
    int64_t* obs;        // OBS: a spread set (zeroed beforehand) that takes (M, E)
    uint32_t xcd_remap;  // renumber blocks per XCD (see logical_block)
    uint32_t nt_store;   // non-temporal stores of the updated rows
};

// STAGED: the wave's lanes own 64 consecutive groups of one row (groups % 64 == 0); rows move
// through LDS with coalesced loads and stores.  Otherwise every lane reads its own 64 bytes, or 32 in
// the half group that ends each row when HALF (L an odd multiple of 32; never STAGED).
template <int Q, bool OBS, bool STAGED, bool HALF = false>
__global__ __launch_bounds__(256) void k_sweep_int8(SweepArgs a) {
    __shared__ uint4 lds_all[4][256];
    const uint32_t lane_id = logical_block(blockIdx.x, gridDim.x, a.xcd_remap) * blockDim.x + threadIdx.x;
    const bool active = lane_id < a.n_lanes;
    Counts cnt{0u, 0u};
    if (active) {
        const uint32_t g = lane_id % a.groups;
        const uint32_t strip = lane_id / a.groups;
        const uint32_t L = a.L;
        const uint32_t r0 = strip * a.rows;
        const uint32_t gl = g == 0 ? a.groups - 1 : g - 1;
        const uint32_t gr = g + 1 == a.groups ? 0 : g + 1;
        const uint32_t lane = threadIdx.x & 63u;
        const bool half = HALF && g + 1 == a.groups;          // this lane's group is a half group
        const uint32_t left_last = HALF && gl + 1 == a.groups ? 28u : 60u;  // last dword of the left group
        uint4* const lds = lds_all[threadIdx.x >> 6];
        // first byte of this lane's group (unstaged) or of the wave's 64 groups (staged)
        int8_t* const col = a.spins + (size_t)(STAGED ? g - lane : g) * 64u;
        auto rowp = [&](uint32_t r) { return col + (size_t)r * L; };
        auto fetch = [&](Row& raw, uint32_t r) {
            if (STAGED) load_row_coalesced(raw, rowp(r), lane);
            else if (half) load_row_half(raw, rowp(r));
            else load_row(raw, rowp(r));
        };
        auto own = [&](Row& row, const Row& raw) {
            if (STAGED) regroup_to_owner(row, raw, lds, lane);
            else row = raw;
        };
        auto put = [&](uint32_t r, const Row& row) {
            if (STAGED) store_row_coalesced(rowp(r), row, lds, lane, a.nt_store);
            else if (half) store_row_half(rowp(r), row);
            else store_row(rowp(r), row, a.nt_store);
        };
        auto halo_left = [&](uint32_t r) {
            return *reinterpret_cast<const uint32_t*>(a.spins + (size_t)r * L + (size_t)gl * 64u + left_last);
        };
        auto halo_right = [&](uint32_t r) {
            return *reinterpret_cast<const uint32_t*>(a.spins + (size_t)r * L + (size_t)gr * 64u);
        };
        auto wrapr = [&](uint32_t r) { return r >= L ? r - L : r; };
        auto halo = [&](uint32_t r, int o) { return o == 1 ? halo_right(r) : halo_left(r); };
        // The horizontal neighbour in the adjacent group: byte 0 of the right group (o = 1) or
        // byte 3 of the left group (o = 0).  When staged, the adjacent groups of row r sit in
        // the neighbouring lanes, so a lane shuffle provides them and only the two lanes at the
        // wave's ends read memory.  (Separate 4-byte loads per lane would reach L2 while the
        // row's own loads are still in flight and fetch every line from DRAM a second time.)
        auto halo_of = [&](const Row& row, uint32_t r, int o) -> uint32_t {
            if (!STAGED) return halo(r, o);
            uint32_t v = o == 1 ? __shfl_down(row.d[0], 1, 64) : __shfl_up(row.d[15], 1, 64);
            if (o == 1 ? lane == 63u : lane == 0u) v = halo(r, o);
            return v;
        };
        // rows r0 (parity offset Q, since r0 is even) and r0 + 1 (offset 1 - Q) alternate.
        // Software pipeline: rows r .. r + 3 and their halo dwords are in registers while
        // rows r + 4, r + 5 are loaded, so HBM latency overlaps two rows of work.
        constexpr int O0 = Q, O1 = 1 - Q;
        // Rows r0 - 1 .. r0 + R are needed (R = a.rows >= 2, even).  Prefetches past r0 + R
        // are clamped to row r0 + R, which is already in cache: the loads stay unconditional
        // so the compiler can keep counting them and never has to drain the memory queue.
        const uint32_t R = a.rows;
        const uint32_t last = r0 + R;
        auto ahead = [&](uint32_t r) { return wrapr(r < last ? r : last); };
        // Pipeline: rows r + 2, r + 3 arrive as raw (coalesced) loads during iteration s - 1 and
        // are regrouped at the top of iteration s, a full iteration after they were requested.
        Row above, cur, nxt, pa, pb, ra, rb;
        fetch(ra, r0 == 0 ? L - 1 : r0 - 1);
        own(above, ra);
        fetch(ra, r0);
        own(cur, ra);
        fetch(ra, wrapr(r0 + 1));
        own(nxt, ra);
        fetch(ra, ahead(r0 + 2));
        fetch(rb, ahead(r0 + 3));
        uint32_t h0 = halo_of(cur, r0, O0), h1 = halo_of(nxt, wrapr(r0 + 1), O1);
        uint32_t bprev = site_bits<O0>(above);
        uint32_t bcur = site_bits<O1>(cur);
#pragma unroll 1
        for (uint32_t s = 0; s < R; s += 2) {
            const uint32_t r = r0 + s;
            own(pa, ra);
            own(pb, rb);
            fetch(ra, ahead(r + 4));
            fetch(rb, ahead(r + 5));
            const uint32_t h2 = halo_of(pa, ahead(r + 2), O0), h3 = halo_of(pb, ahead(r + 3), O1);
            uint32_t bn = sweep_row<Q, O0, OBS>(cur, nxt, bprev, bcur, h0, a.th, g, r, a.t, a.key0, a.key1, cnt, half);
            put(r, cur);
            bprev = bcur;
            bcur = bn;
            bn = sweep_row<Q, O1, OBS>(nxt, pa, bprev, bcur, h1, a.th, g, r + 1, a.t, a.key0, a.key1, cnt, half);
            put(r + 1, nxt);
            bprev = bcur;
            bcur = bn;
            cur = pa;
            nxt = pb;
            h0 = h2;
            h1 = h3;
        }
    }
    // sites in units of 32: a lane covers two per row, one in a half group
    const uint32_t units = !active ? 0u : (HALF && lane_id % a.groups + 1 == a.groups) ? 1u : 2u;
    if (OBS) block_accumulate(spread_line(a.obs, blockIdx.x), cnt.anti, cnt.neg, units, 32u * a.rows);
}

// ---- Fused sweep: both colours of one sweep in one pass over the lattice, out of place.
//
// A workgroup owns a strip of R rows across the full width of the lattice (thread g = column
// group g) and streams down it.  At step x it updates the white sites of row x and then the black
// sites of row x - 1, whose four neighbours (the white sites of rows x - 2, x - 1 and x) are final
// by then.  A white update reads only values the sweep has not changed yet, so the strip also
// recomputes the white sites of the rows just outside it (r0 - 1 and r0 + R) rather than waiting
// for the neighbouring strips: it reads rows r0 - 2 .. r0 + R + 1 of `src` and writes rows
// r0 .. r0 + R - 1 of `dst`.  Every decision takes the same uniform as in the half-sweep kernels,
// so one fused sweep equals a white and then a black half-sweep, bit for bit (Sec. 3.1: sites of
// one colour are independent given the other colour).
//
// Rows are held as two bit words per thread (even and odd columns, site order), so the window of
// four rows costs eight registers.  The neighbour across a group edge comes from the adjacent
// thread through LDS: after step x every thread publishes the edge bits of row x (white sites
// updated) and of row x + 1 (unchanged), and one workgroup barrier per step orders the exchange.
// The barrier fences LDS only, so prefetched row loads and row stores stay in flight across it.
struct FusedArgs {
    const int8_t* src;
    int8_t* dst;
    uint32_t L, groups, rows;  // rows = R, even, divides L; one workgroup per strip of R rows
    uint32_t t, key0, key1;
    Thresholds th;
    int64_t* obs;        // OBS: (M, E) accumulator zeroed beforehand, or a spread set (see spread)
    uint32_t xcd_remap;  // renumber blocks per XCD (see logical_block)
    uint32_t nt_store;   // non-temporal stores of the output rows
    uint32_t alternate;  // walk odd strips upwards
    uint32_t spread;     // k_sweep_fused2q: obs is a spread set (each workgroup adds into its line)
    uint32_t tall;       // k_sweep_fused2p: strips of rows + 2 rows (spread evenly among the others)
};

// Strip l of k_sweep_fused2p (of S = gridDim.x): `tall` of the S strips have rows + 2 rows, the rest
// rows, spread evenly (the first l strips hold floor(l tall / S) tall ones), so that the strips a compute
// unit takes together hold nearly the same number of rows.  Returns the strip's first row and sets R.
__device__ __forceinline__ uint32_t pair_strip_rows(uint32_t l, uint32_t S, uint32_t rows, uint32_t tall,
                                                    uint32_t& R) {
    const uint32_t before = (uint32_t)(((uint64_t)l * tall) / S);
    const uint32_t upto = (uint32_t)(((uint64_t)(l + 1u) * tall) / S);
    R = rows + 2u * (upto - before);
    return l * rows + 2u * before;
}

// Edge bits a thread publishes after step x: bit 0 / 1 = site 0 of the even columns / site 31 of
// the odd columns of row x + 1, bit 2 / 3 = the same sites of row x.
__device__ __forceinline__ uint32_t edge_word(const RowBits& next, const RowBits& cur) {
    return (next.e & 1u) | ((next.o >> 31) << 1) | ((cur.e & 1u) << 2) | ((cur.o >> 31) << 3);
}

// One step at row x: the white sites of row x (w0), then, with B, the black sites of row x - 1 (w1).
// O = column parity of row x's white sites, which is also that of row x - 1's black sites.
// w2 = row x - 2, wn = row x + 1; nb = the edge word of the right neighbour group (O = 1) or of the
// left one (O = 0), published after step x - 1.
template <int O, bool B, bool OBS>
__device__ __forceinline__ void fused_step(const RowBits& w2, RowBits& w1, RowBits& w0, const RowBits& wn, uint32_t nb,
                                           const Thresholds& th, uint32_t g, uint32_t x, uint32_t xm1, uint32_t t,
                                           uint32_t key0, uint32_t key1, Counts& cnt) {
    {
        const uint32_t side = O ? w0.e : w0.o;
        const uint32_t hs = O ? shift_next(side, nb & 1u) : shift_prev(side, (nb >> 1) & 1u);
        const uint32_t F = decide<1, false>(O ? w0.o : w0.e, O ? w1.o : w1.e, O ? wn.o : wn.e, side, hs, 0u, th, g,
                                            x, t, key0, key1, cnt);
        if (O) w0.o ^= F; else w0.e ^= F;
    }
    if (B) {
        const uint32_t side = O ? w1.e : w1.o;
        const uint32_t hs = O ? shift_next(side, (nb >> 2) & 1u) : shift_prev(side, (nb >> 3) & 1u);
        const uint32_t F = decide<0, OBS>(O ? w1.o : w1.e, O ? w2.o : w2.e, O ? w0.o : w0.e, side, hs, side, th, g,
                                          xm1, t, key0, key1, cnt);
        if (O) w1.o ^= F; else w1.e ^= F;
    }
}

// One strip of the fused sweep.  UP: the strip is walked from its last row to its first (the
// same updates in mirror order: white sites of row x, then black sites of row x + 1).  Strips
// alternate direction so that two neighbouring strips read the rows around their common boundary
// at the same time (both at the end, or both at the start), and the second read hits in L2.
// STAGED: groups % 64 == 0 and every wave moves its 64 groups' rows with coalesced loads and
// stores through LDS; otherwise every thread reads and writes its own 64 bytes, and threads past
// the last group shadow it without storing (they still take part in the barriers).
template <bool OBS, bool STAGED, bool UP>
__device__ __forceinline__ void fused_strip(const FusedArgs& a, uint32_t strip, uint4* fused_lds, Counts& cnt) {
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    const uint32_t G = a.groups, L = a.L, R = a.rows;
    uint4* const stage = fused_lds + (tid >> 6) * 256u;  // STAGED: 4 KiB per wave
    uint32_t* const xch = reinterpret_cast<uint32_t*>(fused_lds + (STAGED ? (nt >> 6) * 256u : 0u));
    const bool active = tid < G;
    const uint32_t g = active ? tid : G - 1;
    const uint32_t gl = g == 0 ? G - 1 : g - 1, gr = g + 1 == G ? 0 : g + 1;
    const uint32_t lane = tid & 63u;
    const uint32_t r0 = __builtin_amdgcn_readfirstlane(strip * R);  // uniform: keeps the row arithmetic scalar
    const size_t col = (size_t)(STAGED ? g - lane : g) * 64u;
    // k-th row of the walk, k = 0 .. R + 3: r0 - 2 .. r0 + R + 1 (down) or r0 + R + 1 .. r0 - 2
    // (up), wrapped onto the torus.  Prefetches past the walk's last row are clamped to it (already
    // in cache), so every load stays unconditional.
    auto vrow = [&](uint32_t k) {
        const uint32_t kk = k < R + 3 ? k : R + 3;
        const uint32_t v = UP ? r0 + R + 1 + L - kk : r0 + L + kk - 2;  // in [L - 2, 2L + 2)
        return v >= 2 * L ? v - 2 * L : v >= L ? v - L : v;
    };
    auto fetch = [&](Row& raw, uint32_t r) {
        if (STAGED) load_row_coalesced(raw, a.src + (size_t)r * L + col, lane);
        else load_row(raw, a.src + (size_t)r * L + col);
    };
    auto own = [&](const Row& raw) {
        if (!STAGED) return row_bits(raw);
        Row row;
        regroup_to_owner(row, raw, stage, lane);
        return row_bits(row);
    };
    auto put = [&](uint32_t r, const RowBits& b) {
        Row row;
        bits_to_row(row, b);
        if (STAGED) store_row_coalesced(a.dst + (size_t)r * L + col, row, stage, lane, a.nt_store);
        else if (active) store_row(a.dst + (size_t)r * L + col, row, a.nt_store);
    };
    // The white sites of walk row k + 1 lie on columns of parity OA for even k, OB for odd k
    // (r0 and R are even).  A step with parity 1 takes the edge word of the right neighbour
    // group, one with parity 0 that of the left one; step k reads slot (k + 1) & 1.
    constexpr int OA = UP ? 1 : 0, OB = 1 - OA;
    const uint32_t nbA = OA ? gr : gl, nbB = OB ? gr : gl;
    const uint32_t t = a.t, k0 = a.key0, k1 = a.key1;
    // prologue: walk rows 0 .. 3 in bits, rows 4, 5 in flight
    // (two row buffers throughout, which keeps the register count at four waves per SIMD)
    Row ra, rb;
    fetch(ra, vrow(0));
    fetch(rb, vrow(1));
    RowBits w2{0u, 0u};
    RowBits w1 = own(ra), w0 = own(rb);
    fetch(ra, vrow(2));
    fetch(rb, vrow(3));
    RowBits n0 = own(ra), n1 = own(rb);
    fetch(ra, vrow(4));
    fetch(rb, vrow(5));
    xch[nt + tid] = edge_word(w0, w0);  // slot 1: walk row 1 (bits 2, 3 unused)
    workgroup_lds_sync();
    // walk rows 1 and 2: white sites only (walk row 1 belongs to the neighbouring strip)
    fused_step<OA, false, false>(w2, w1, w0, n0, xch[nt + nbA], a.th, g, vrow(1), 0u, t, k0, k1, cnt);
    xch[tid] = edge_word(n0, w0);
    workgroup_lds_sync();
    w2 = w1; w1 = w0; w0 = n0;
    fused_step<OB, false, false>(w2, w1, w0, n1, xch[nbB], a.th, g, vrow(2), 0u, t, k0, k1, cnt);
    xch[nt + tid] = edge_word(n1, w0);
    workgroup_lds_sync();
    w2 = w1; w1 = w0; w0 = n1;
    n0 = own(ra);
    n1 = own(rb);
    fetch(ra, vrow(6));
    fetch(rb, vrow(7));
    // Rows are regrouped at the end of the iteration after the one that requested them, behind
    // that iteration's stores: the wait for a row's loads then leaves the stores in flight, and
    // every path into the loop head has the same memory operations outstanding.
#pragma unroll 1
    for (uint32_t k = 2; k < R + 2; k += 2) {
        // steps k, k + 1: white sites of walk rows k + 1, k + 2, black sites of walk rows k, k + 1
        fused_step<OA, true, OBS>(w2, w1, w0, n0, xch[nt + nbA], a.th, g, vrow(k + 1), vrow(k), t, k0, k1, cnt);
        put(vrow(k), w1);
        xch[tid] = edge_word(n0, w0);
        workgroup_lds_sync();
        w2 = w1; w1 = w0; w0 = n0;
        fused_step<OB, true, OBS>(w2, w1, w0, n1, xch[nbB], a.th, g, vrow(k + 2), vrow(k + 1), t, k0, k1, cnt);
        put(vrow(k + 1), w1);
        xch[nt + tid] = edge_word(n1, w0);
        workgroup_lds_sync();
        w2 = w1; w1 = w0; w0 = n1;
        n0 = own(ra);  // walk rows k + 4, k + 5 for the next iteration
        n1 = own(rb);
        fetch(ra, vrow(k + 6));
        fetch(rb, vrow(k + 7));
    }
}

template <bool OBS, bool STAGED>
__global__ __launch_bounds__(1024) void k_sweep_fused(FusedArgs a) {
    extern __shared__ uint4 fused_lds[];
    const uint32_t strip = logical_block(blockIdx.x, gridDim.x, a.xcd_remap);
    Counts cnt{0u, 0u};
    if (a.alternate && (strip & 1u)) fused_strip<OBS, STAGED, true>(a, strip, fused_lds, cnt);
    else fused_strip<OBS, STAGED, false>(a, strip, fused_lds, cnt);
    const bool active = threadIdx.x < a.groups;
    if (OBS) block_accumulate(a.obs, active ? cnt.anti : 0u, active ? cnt.neg : 0u, active ? 1u : 0u, 64u * a.rows);
}


// ---- Two sweeps per pass: sweeps t and t + 1 in one walk down the strip.
//
// The walk of the one-sweep pass extended by one lagging row per colour update: at step x the
// strip updates the white sites of row x (sweep t), the black sites of row x - 1 (sweep t), the
// white sites of row x - 2 (sweep t + 1) and the black sites of row x - 3 (sweep t + 1).  Each
// update finds its neighbours final for its sweep (the row below it was updated one update
// earlier in the same step, the row above one step earlier), and all four share one column
// parity, so one edge word per step (two bits per row, four rows) carries every horizontal
// neighbour across a group edge.  The strip recomputes the rows its neighbours own that its own
// rows depend on: it reads rows r0 - 4 .. r0 + R + 3, updates white sites of rows r0 - 3 ..
// r0 + R + 2 and r0 - 1 .. r0 + R and black sites of rows r0 - 2 .. r0 + R + 1 and r0 ..
// r0 + R - 1, and writes rows r0 .. r0 + R - 1 after sweep t + 1.  The result is two fused
// sweeps, bit for bit.

// Edge bits after a step: bits 2k, 2k + 1 = site 0 of the even columns and site 31 of the odd
// columns of the k-th row (k = 0: the next row to be updated; then the updated rows below it).
__device__ __forceinline__ uint32_t edge_word4(const RowBits& r0, const RowBits& r1, const RowBits& r2,
                                               const RowBits& r3) {
    return (r0.e & 1u) | ((r0.o >> 31) << 1) | ((r1.e & 1u) << 2) | ((r1.o >> 31) << 3) | ((r2.e & 1u) << 4) |
           ((r2.o >> 31) << 5) | ((r3.e & 1u) << 6) | ((r3.o >> 31) << 7);
}

// One colour-Q update of the sites of `own` at column parity O; v0 / v1 = the rows on either side;
// P = which bit pair of the edge word holds this row's neighbour across the group edge.  With
// OBS and `count`, the sites' anti-aligned bonds and the row's -1 spins go to cnt.
template <int O, int Q, int P, bool OBS>
__device__ __forceinline__ void fused_update(RowBits& own, const RowBits& v0, const RowBits& v1, uint32_t nb,
                                             const Thresholds& th, uint32_t g, uint32_t row, uint32_t t,
                                             uint32_t key0, uint32_t key1, Counts& cnt, bool count) {
    const uint32_t side = O ? own.e : own.o;
    const uint32_t hs = O ? shift_next(side, (nb >> (2 * P)) & 1u) : shift_prev(side, (nb >> (2 * P + 1)) & 1u);
    Counts c{0u, 0u};
    const uint32_t F = decide<Q, OBS>(O ? own.o : own.e, O ? v0.o : v0.e, O ? v1.o : v1.e, side, hs,
                                      Q == 0 ? side : 0u, th, g, row, t, key0, key1, c);
    if (OBS && count) { cnt.anti += c.anti; cnt.neg += c.neg; }
    if (O) own.o ^= F; else own.e ^= F;
}

// One step of the two-sweep walk with the first NU of its four updates (the walk's first steps
// have rows below them that are not there yet).  w0 = the row of the white update of sweep t, w1
// .. w4 the rows after it, wn the row before it; rows[k] = global row of update k.
template <int O, int NU, bool OBS>
__device__ __forceinline__ void fused2_step(RowBits& w4, RowBits& w3, RowBits& w2, RowBits& w1, RowBits& w0,
                                            const RowBits& wn, uint32_t nb, const Thresholds& th, uint32_t g,
                                            const uint32_t (&rows)[4], uint32_t t, uint32_t key0, uint32_t key1,
                                            Counts& ct, Counts& ct1, bool count_t) {
    fused_update<O, 1, 0, false>(w0, w1, wn, nb, th, g, rows[0], t, key0, key1, ct, false);
    if (NU >= 2) fused_update<O, 0, 1, OBS>(w1, w2, w0, nb, th, g, rows[1], t, key0, key1, ct, count_t);
    if (NU >= 3) fused_update<O, 1, 2, false>(w2, w3, w1, nb, th, g, rows[2], t + 1, key0, key1, ct1, false);
    if (NU >= 4) fused_update<O, 0, 3, OBS>(w3, w4, w2, nb, th, g, rows[3], t + 1, key0, key1, ct1, true);
}

template <bool OBS, bool STAGED, bool UP>
__device__ __forceinline__ void fused2_strip(const FusedArgs& a, uint32_t strip, uint4* fused_lds, Counts& ct,
                                             Counts& ct1) {
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    const uint32_t G = a.groups, L = a.L, R = a.rows;
    uint4* const stage = fused_lds + (tid >> 6) * 256u;  // STAGED: 4 KiB per wave
    uint32_t* const xch = reinterpret_cast<uint32_t*>(fused_lds + (STAGED ? (nt >> 6) * 256u : 0u));
    const bool active = tid < G;
    const uint32_t g = active ? tid : G - 1;
    const uint32_t gl = g == 0 ? G - 1 : g - 1, gr = g + 1 == G ? 0 : g + 1;
    const uint32_t lane = tid & 63u;
    const uint32_t r0 = __builtin_amdgcn_readfirstlane(strip * R);  // uniform: keeps the row arithmetic scalar
    const size_t col = (size_t)(STAGED ? g - lane : g) * 64u;
    // walk row k = 0 .. R + 7: r0 - 4 .. r0 + R + 3 (down) or r0 + R + 3 .. r0 - 4 (up), wrapped
    // onto the torus; prefetches past the last walk row are clamped to it
    auto vrow = [&](uint32_t k) {
        const uint32_t kk = k < R + 7 ? k : R + 7;
        // in [-4, L + 4) since r0 + R <= L; signed compares keep the wrap on the scalar unit
        const int32_t v = (int32_t)(UP ? r0 + R + 3 - kk : r0 + kk) - (UP ? 0 : 4);
        return (uint32_t)(v < 0 ? v + (int32_t)L : v >= (int32_t)L ? v - (int32_t)L : v);
    };
    auto fetch = [&](Row& raw, uint32_t r) {
        if (STAGED) load_row_coalesced(raw, a.src + (size_t)r * L + col, lane);
        else load_row(raw, a.src + (size_t)r * L + col);
    };
    auto own = [&](const Row& raw) {
        if (!STAGED) return row_bits(raw);
        Row row;
        regroup_to_owner(row, raw, stage, lane);
        return row_bits(row);
    };
    auto put = [&](uint32_t r, const RowBits& b) {
        Row row;
        bits_to_row(row, b);
        if (STAGED) store_row_coalesced(a.dst + (size_t)r * L + col, row, stage, lane, a.nt_store);
        else if (active) store_row(a.dst + (size_t)r * L + col, row, a.nt_store);
    };
    // step s (s = 0 .. R + 5) updates walk rows s + 1 (white, t), s (black, t), s - 1 (white,
    // t + 1), s - 2 (black, t + 1); its sites lie on columns of parity OA for even s, OB for odd s.
    // A step with parity 1 takes the edge word of the right neighbour group, one with parity 0
    // that of the left one; step s reads slot s & 1 and publishes into the other.
    constexpr int OA = UP ? 1 : 0, OB = 1 - OA;
    const uint32_t nbA = OA ? gr : gl, nbB = OB ? gr : gl;
    const uint32_t t = a.t, k0 = a.key0, k1 = a.key1;
    Row ra, rb;
    fetch(ra, vrow(0));
    fetch(rb, vrow(1));
    RowBits w4{0u, 0u}, w3{0u, 0u}, w2{0u, 0u};
    RowBits w1 = own(ra), w0 = own(rb);
    fetch(ra, vrow(2));
    fetch(rb, vrow(3));
    RowBits n0 = own(ra), n1 = own(rb);
    fetch(ra, vrow(4));
    fetch(rb, vrow(5));
    xch[tid] = edge_word4(w0, w1, w1, w1);  // slot 0: walk row 1 (the other pairs are not read)
    workgroup_lds_sync();
#define ISING_FUSED2_STEP(O, NU, NB, S, NEXT)                                                                 \
    do {                                                                                                      \
        const uint32_t s_ = (S);                                                                              \
        const uint32_t rw[4] = {vrow(s_ + 1), vrow(s_), s_ >= 1 ? vrow(s_ - 1) : 0u, s_ >= 2 ? vrow(s_ - 2) : 0u}; \
        fused2_step<O, NU, OBS>(w4, w3, w2, w1, w0, NEXT, xch[(s_ & 1u) * nt + (NB)], a.th, g, rw, t, k0, k1, ct, \
                                ct1, s_ >= 4 && s_ <= R + 3);                                                 \
        if (NU == 4) put(rw[3], w3);                                                                          \
        xch[((s_ + 1) & 1u) * nt + tid] = edge_word4(NEXT, w0, w1, w2);                                       \
        workgroup_lds_sync();                                                                                 \
        w4 = w3; w3 = w2; w2 = w1; w1 = w0; w0 = NEXT;                                                        \
    } while (0)
    // steps 0 .. 5: the updates that have rows below them
    ISING_FUSED2_STEP(OA, 1, nbA, 0u, n0);
    ISING_FUSED2_STEP(OB, 1, nbB, 1u, n1);
    n0 = own(ra);
    n1 = own(rb);
    fetch(ra, vrow(6));
    fetch(rb, vrow(7));
    ISING_FUSED2_STEP(OA, 2, nbA, 2u, n0);
    ISING_FUSED2_STEP(OB, 2, nbB, 3u, n1);
    n0 = own(ra);
    n1 = own(rb);
    fetch(ra, vrow(8));
    fetch(rb, vrow(9));
    ISING_FUSED2_STEP(OA, 3, nbA, 4u, n0);
    ISING_FUSED2_STEP(OB, 3, nbB, 5u, n1);
    n0 = own(ra);
    n1 = own(rb);
    fetch(ra, vrow(10));
    fetch(rb, vrow(11));
    // steps 6 .. R + 5: all four updates, and the row of the last one is final
#pragma unroll 1
    for (uint32_t s = 6; s < R + 6; s += 2) {
        ISING_FUSED2_STEP(OA, 4, nbA, s, n0);
        ISING_FUSED2_STEP(OB, 4, nbB, s + 1, n1);
        n0 = own(ra);  // walk rows s + 4, s + 5 for the next two steps
        n1 = own(rb);
        fetch(ra, vrow(s + 6));
        fetch(rb, vrow(s + 7));
    }
#undef ISING_FUSED2_STEP
}

template <bool OBS, bool STAGED>
__global__ __launch_bounds__(1024) void k_sweep_fused2(FusedArgs a) {
    extern __shared__ uint4 fused_lds[];
    const uint32_t strip = logical_block(blockIdx.x, gridDim.x, a.xcd_remap);
    Counts ct{0u, 0u}, ct1{0u, 0u};
    if (a.alternate && (strip & 1u)) fused2_strip<OBS, STAGED, true>(a, strip, fused_lds, ct, ct1);
    else fused2_strip<OBS, STAGED, false>(a, strip, fused_lds, ct, ct1);
    const bool active = threadIdx.x < a.groups;
    if (OBS) {
        block_accumulate(a.obs, active ? ct.anti : 0u, active ? ct.neg : 0u, active ? 1u : 0u, 64u * a.rows);
        __syncthreads();  // block_accumulate's LDS is reused
        block_accumulate(a.obs + 2, active ? ct1.anti : 0u, active ? ct1.neg : 0u, active ? 1u : 0u, 64u * a.rows);
    }
}

// ---- Two sweeps per pass, with the ties of a step settled together.
//
// In the walk above each update needs the result of the one before it in the same step, so each
// waits for the last undecided site of its wave: a word costs about 3.3 Philox blocks, where one
// site needs about 1.07 on average (15 of 16 sites are decided by the first four bit planes).
// This walk leaves two rows between consecutive updates: step s updates the white sites of walk
// row s + 1 (sweep t), the black sites of s - 1 (t), the white sites of s - 3 (t + 1) and the
// black sites of s - 5 (t + 1).  Every value an update reads was final at the end of step s - 1
// and no update of the step writes it, so the four updates of a step are independent.  Each
// takes its first two Philox blocks (eight bit planes) for all its sites; a word with sites still
// tied after that goes to a queue in the wave's LDS, and the wave then settles the queued words
// of all four updates at once, one word per lane.  About 25 words are queued per step, so the
// planes after the eighth cost about two blocks per step instead of about 1.3 per update.  The
// strip reads, recomputes and writes the same rows as the walk above, and every decision takes
// the same uniform, so the result is the same two sweeps, bit for bit.

// One colour-Q update at column parity O (P = its pair in the edge words): the sites decided by
// the first two Philox blocks flip at once, the word's remaining ties go to the queue (n entries,
// uniform).  nbL / nbR = the edge words of the left / right neighbour group.
template <int O, int Q, int P>
__device__ __forceinline__ void tq_update(RowBits& own, const RowBits& v0, const RowBits& v1, uint32_t nbL,
                                          uint32_t nbR, const Thresholds& th, uint32_t g, uint32_t row, uint32_t t,
                                          uint32_t key0, uint32_t key1, const TieQueue& q, uint32_t& n,
                                          uint32_t lane) {
    const uint32_t side = O ? own.e : own.o;
    const uint32_t hs = O ? shift_next(side, (nbR >> (2 * P)) & 1u) : shift_prev(side, (nbL >> (2 * P + 1)) & 1u);
    const uint32_t a = O ? own.o : own.e;
    const uint32_t x1 = a ^ (O ? v0.o : v0.e), x2 = a ^ (O ? v1.o : v1.e), x3 = a ^ side, x4 = a ^ hs;
    const uint32_t o12 = x1 | x2, o34 = x3 | x4;
    const uint32_t ge2 = (x1 & x2) | (x3 & x4) | (o12 & o34);  // s <= 0: always flips
    const uint32_t any = o12 | o34;
    // sites that flip without a uniform: s <= 0, and s = 2 / s = 4 where T_s = 2^32 (uniform masks)
    const uint32_t flip = (ge2 | (any & th.f2)) | (~any & th.f4);
    const uint32_t sel2 = any & ~flip;
    uint32_t acc = flip, tied = ~flip;
    // the row is the same for the whole wave: keeping it in a scalar register lets the Philox rounds
    // that depend only on (row, sweep, colour) run on the scalar unit
    const uint32_t urow = __builtin_amdgcn_readfirstlane(row);
#pragma unroll
    for (uint32_t m = 0; m < 2; ++m) {
        if (!wave_any(tied != 0u)) break;
        compare_planes(acc, tied, sel2, philox4x32_10<2, 3>(g, urow, t, 2u * m + (uint32_t)Q, key0, key1), th, m);
    }
    if (O) own.o ^= acc; else own.e ^= acc;
    tq_push(q, n, tied, sel2, row, (uint32_t)P | (lane << 2) | (g << 8));
}

// (M, E) contributions of the colour sites of `own` at parity O after their update (P as in
// tq_update): their anti-aligned bonds, and the -1 spins of both colours of the row.
template <int O, int P>
__device__ __forceinline__ void tq_count(const RowBits& own, const RowBits& v0, const RowBits& v1, uint32_t nbL,
                                         uint32_t nbR, Counts& cnt) {
    const uint32_t side = O ? own.e : own.o;
    const uint32_t hs = O ? shift_next(side, (nbR >> (2 * P)) & 1u) : shift_prev(side, (nbL >> (2 * P + 1)) & 1u);
    const uint32_t a = O ? own.o : own.e;
    cnt.anti += __builtin_popcount(a ^ (O ? v0.o : v0.e)) + __builtin_popcount(a ^ (O ? v1.o : v1.e)) +
                __builtin_popcount(a ^ side) + __builtin_popcount(a ^ hs);
    cnt.neg += __builtin_popcount(a) + __builtin_popcount(side);
}

// One step s of the walk: U1 (white, t) on w0 between wn and w1, U2 (black, t) on w2, U3 (white,
// t + 1) on w4, U4 (black, t + 1) on w6.  U1 and U3 lie on columns of parity O, U2 and U4 on 1 - O.
// rows[k] = global row of update k; act = which updates the step makes (bit k: update k);
// count_t: U2's row is one the strip writes.
template <int O, bool OBS>
__device__ __forceinline__ void fused2q_step(RowBits& w0, RowBits& w2, RowBits& w4, RowBits& w6, const RowBits& wn,
                                             const RowBits& w1, const RowBits& w3, const RowBits& w5,
                                             const RowBits& w7, uint32_t nbL, uint32_t nbR, const Thresholds& th,
                                             uint32_t g, const uint32_t (&rows)[4], uint32_t act, uint32_t t,
                                             uint32_t key0, uint32_t key1, const TieQueue& q, uint32_t lane,
                                             Counts& ct, Counts& ct1, bool count_t) {
    constexpr int X = 1 - O;
    q.res[lane] = make_uint4(0u, 0u, 0u, 0u);
    uint32_t n = 0u;
    if (act & 1u) tq_update<O, 1, 0>(w0, wn, w1, nbL, nbR, th, g, rows[0], t, key0, key1, q, n, lane);
    if (act & 2u) tq_update<X, 0, 1>(w2, w1, w3, nbL, nbR, th, g, rows[1], t, key0, key1, q, n, lane);
    if (act & 4u) tq_update<O, 1, 2>(w4, w3, w5, nbL, nbR, th, g, rows[2], t + 1u, key0, key1, q, n, lane);
    if (act & 8u) tq_update<X, 0, 3>(w6, w5, w7, nbL, nbR, th, g, rows[3], t + 1u, key0, key1, q, n, lane);
    tq_settle<-1>(q, n, th, t, key0, key1, lane);
    const uint4 r = q.res[lane];  // zero for the updates the step does not make
    if (O) { w0.o ^= r.x; w4.o ^= r.z; w2.e ^= r.y; w6.e ^= r.w; }
    else { w0.e ^= r.x; w4.e ^= r.z; w2.o ^= r.y; w6.o ^= r.w; }
    if (OBS) {
        if ((act & 2u) && count_t) tq_count<X, 1>(w2, w1, w3, nbL, nbR, ct);
        if (act & 8u) tq_count<X, 3>(w6, w5, w7, nbL, nbR, ct1);
    }
}

template <bool OBS, bool STAGED, bool UP>
__device__ __forceinline__ void fused2q_strip(const FusedArgs& a, uint32_t strip, uint4* fused_lds, Counts& ct,
                                              Counts& ct1) {
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    const uint32_t G = a.groups, L = a.L, R = a.rows;
    // 5 KiB per wave: row staging (4 KiB) shared with the tie queue's entries, and its results
    uint4* const stage = fused_lds + (tid >> 6) * (kTieQueueBytes / 16u);
    uint32_t* const xch = reinterpret_cast<uint32_t*>(fused_lds + (nt >> 6) * (kTieQueueBytes / 16u));
    const TieQueue q{reinterpret_cast<uint32_t*>(stage), stage + 256};
    const bool active = tid < G;
    const uint32_t g = active ? tid : G - 1;
    const uint32_t gl = g == 0 ? G - 1 : g - 1, gr = g + 1 == G ? 0 : g + 1;
    const uint32_t lane = tid & 63u;
    const uint32_t r0 = __builtin_amdgcn_readfirstlane(strip * R);  // uniform: keeps the row arithmetic scalar
    const size_t col = (size_t)(STAGED ? g - lane : g) * 64u;
    // walk row k = 0 .. R + 7: r0 - 4 .. r0 + R + 3 (down) or r0 + R + 3 .. r0 - 4 (up), wrapped
    // onto the torus; prefetches past the last walk row are clamped to it
    auto vrow = [&](uint32_t k) {
        const uint32_t kk = k < R + 7 ? k : R + 7;
        // in [-4, L + 4) since r0 + R <= L; signed compares keep the wrap on the scalar unit
        const int32_t v = (int32_t)(UP ? r0 + R + 3 - kk : r0 + kk) - (UP ? 0 : 4);
        return (uint32_t)(v < 0 ? v + (int32_t)L : v >= (int32_t)L ? v - (int32_t)L : v);
    };
    auto fetch = [&](Row& raw, uint32_t r) {
        if (STAGED) load_row_coalesced(raw, a.src + (size_t)r * L + col, lane);
        else load_row(raw, a.src + (size_t)r * L + col);
    };
    auto own = [&](const Row& raw) {
        if (!STAGED) return row_bits(raw);
        Row row;
        regroup_to_owner(row, raw, stage, lane);
        return row_bits(row);
    };
    auto put = [&](uint32_t r, const RowBits& b) {
        Row row;
        bits_to_row(row, b);
        if (STAGED) store_row_coalesced(a.dst + (size_t)r * L + col, row, stage, lane, a.nt_store);
        else if (active) store_row(a.dst + (size_t)r * L + col, row, a.nt_store);
    };
    // Step s (s = 0 .. R + 8) makes U1 for s <= R + 5 (walk rows 1 .. R + 6), U2 for 3 <= s <= R + 6
    // (rows 2 .. R + 5), U3 for 6 <= s <= R + 7 (rows 3 .. R + 4) and U4 for 9 <= s <= R + 8 (rows
    // 4 .. R + 3, the strip's own rows, written after their update).  U1 and U3 of an even step lie
    // on columns of parity OA.  Step s reads edge-word slot s & 1 and publishes into the other.
    constexpr int OA = UP ? 1 : 0, OB = 1 - OA;
    const uint32_t t = a.t, k0 = a.key0, k1 = a.key1;
    // one prefetched row in flight: the row a step needs next is requested a step ahead
    Row raw;
    fetch(raw, vrow(0));
    RowBits w7{0u, 0u}, w6{0u, 0u}, w5{0u, 0u}, w4{0u, 0u}, w3{0u, 0u}, w2{0u, 0u};
    RowBits w1 = own(raw);
    fetch(raw, vrow(1));
    RowBits w0 = own(raw);
    fetch(raw, vrow(2));
    RowBits nx = own(raw);
    fetch(raw, vrow(3));
    xch[tid] = edge_word4(w0, w2, w4, w6);  // slot 0: walk row 1 (the other pairs are not read)
    workgroup_lds_sync();
#define ISING_FUSED2Q_STEP(O, S)                                                                             \
    do {                                                                                                     \
        const uint32_t s_ = (S);                                                                             \
        const uint32_t act = (s_ <= R + 5 ? 1u : 0u) | (s_ >= 3 && s_ <= R + 6 ? 2u : 0u) |                 \
                             (s_ >= 6 && s_ <= R + 7 ? 4u : 0u) | (s_ >= 9 && s_ <= R + 8 ? 8u : 0u);        \
        const uint32_t rw[4] = {vrow(s_ + 1), s_ >= 1 ? vrow(s_ - 1) : 0u, s_ >= 3 ? vrow(s_ - 3) : 0u,      \
                                s_ >= 5 ? vrow(s_ - 5) : 0u};                                                \
        const uint32_t sl = (s_ & 1u) * nt;                                                                  \
        fused2q_step<O, OBS>(w0, w2, w4, w6, nx, w1, w3, w5, w7, xch[sl + gl], xch[sl + gr], a.th, g, rw,    \
                             act, t, k0, k1, q, lane, ct, ct1, s_ >= 5 && s_ <= R + 4);                       \
        if (act & 8u) put(rw[3], w6);                                                                        \
        w7 = w6; w6 = w5; w5 = w4; w4 = w3; w3 = w2; w2 = w1; w1 = w0; w0 = nx;                              \
        xch[((s_ + 1) & 1u) * nt + tid] = edge_word4(w0, w2, w4, w6);                                        \
        nx = own(raw);  /* walk row s + 3 */                                                                 \
        fetch(raw, vrow(s_ + 4));                                                                            \
        workgroup_lds_sync();                                                                                \
    } while (0)
#pragma unroll 1
    for (uint32_t s = 0; s < R + 10; s += 2) {  // step R + 9 makes no update
        ISING_FUSED2Q_STEP(OA, s);
        ISING_FUSED2Q_STEP(OB, s + 1);
    }
#undef ISING_FUSED2Q_STEP
}

template <bool OBS, bool STAGED>
__global__ __launch_bounds__(1024) void k_sweep_fused2q(FusedArgs a) {
    extern __shared__ uint4 fused_lds[];
    const uint32_t strip = logical_block(blockIdx.x, gridDim.x, a.xcd_remap);
    Counts ct{0u, 0u}, ct1{0u, 0u};
    if (a.alternate && (strip & 1u)) fused2q_strip<OBS, STAGED, true>(a, strip, fused_lds, ct, ct1);
    else fused2q_strip<OBS, STAGED, false>(a, strip, fused_lds, ct, ct1);
    const bool active = threadIdx.x < a.groups;
    if (OBS) {
        int64_t* const out = a.spread ? spread_line(a.obs, blockIdx.x) : a.obs;
        block_accumulate(out, active ? ct.anti : 0u, active ? ct.neg : 0u, active ? 1u : 0u, 64u * a.rows);
        __syncthreads();  // block_accumulate's LDS is reused
        block_accumulate(out + 2, active ? ct1.anti : 0u, active ? ct1.neg : 0u, active ? 1u : 0u, 64u * a.rows);
    }
}

// ---- Two sweeps per pass, the ties of two steps settled together.
//
// The walk of the pass above with three rows between its updates instead of two: step s updates the
// white sites of walk row s + 1 (sweep t), the black sites of s - 2 (t), the white sites of s - 5
// (t + 1) and the black sites of s - 8 (t + 1).  Each update reads only rows that the updates of
// steps s - 2 and earlier have finished (the neighbours of a black update of sweep t are white sites
// of sweep t two, three and four steps back, and so on down the chain of Sec. 3.1's colour updates),
// and no update of step s + 1 reads a row that step s writes.  So the eight updates of an even step
// and the step after it are independent: they share one edge exchange, one workgroup barrier and
// one settle of the wave's tie queue (about twice as many queued words per settle, so fewer Philox
// blocks past the eighth plane).  The strip reads, recomputes and writes the same rows as the pass
// above, and every decision takes the same uniform, so the result is the same two sweeps, bit for
// bit.  Two waves per SIMD (up to 256 registers): each update draws its first two Philox blocks as
// two independent chains, and the next two walk rows are fetched a pair ahead.

constexpr uint32_t kPairQueueCap = 512;                        // 8 updates x 64 lanes
constexpr uint32_t kPairQueueSlots = kPairQueueCap + 64u;       // and one write-off slot per lane
constexpr uint32_t kPairWaveBytes = kPairQueueSlots * 16u + 8u * 64u * 4u;  // 9 KiB entries, 2 KiB results

// Per-wave LDS of the pair's tie queue: task[576] = (tied, tied & sel2, Philox row, meta = u | lane << 3 |
// group << 9), one 16-byte entry each, and res[8][64] = the sites of update u of lane l that the queue
// accepted (update-major, so that neither the settle's scattered writes nor a lane's reads collide on
// LDS banks).  A lane with no tied site writes its entry to its own slot past the queue (512 + lane), so
// that a push is straight-line code.  The first 4 KiB double as the row staging buffer outside the pushes
// and the settle.
struct PairQueue {
    uint4* task;
    uint32_t* res;
};

// Edge bits of the pair's eight update rows (2U, 2U + 1: site 0 of the even columns and site 31 of the
// odd columns of update U's row), taken when the pair starts.
__device__ __forceinline__ uint32_t pair_edges(const RowBits& r0, const RowBits& r1, const RowBits& r2,
                                               const RowBits& r3, const RowBits& r4, const RowBits& r5,
                                               const RowBits& r6, const RowBits& r7) {
    return edge_word4(r0, r1, r2, r3) | (edge_word4(r4, r5, r6, r7) << 8);
}

// Update U (0 .. 7) of a pair: colour Q at column parity O of `own` between v0 and v1; sweep t is the
// update's own.  The first two Philox blocks decide at once; words still tied go to the queue.
template <int O, int Q, int U>
__device__ __forceinline__ void pair_update(RowBits& own, const RowBits& v0, const RowBits& v1, uint32_t nbL,
                                            uint32_t nbR, const Thresholds& th, uint32_t g, uint32_t row, uint32_t t,
                                            uint32_t key0, uint32_t key1, const PairQueue& q, uint32_t& n,
                                            uint32_t lane) {
    const uint32_t side = O ? own.e : own.o;
    const uint32_t hs = O ? shift_next(side, (nbR >> (2 * U)) & 1u) : shift_prev(side, (nbL >> (2 * U + 1)) & 1u);
    const uint32_t a = O ? own.o : own.e;
    const uint32_t x1 = a ^ (O ? v0.o : v0.e), x2 = a ^ (O ? v1.o : v1.e), x3 = a ^ side, x4 = a ^ hs;
    const uint32_t o12 = x1 | x2, o34 = x3 | x4;
    const uint32_t ge2 = (x1 & x2) | (x3 & x4) | (o12 & o34);  // s <= 0: always flips
    const uint32_t any = o12 | o34;
    const uint32_t flip = (ge2 | (any & th.f2)) | (~any & th.f4);
    const uint32_t sel2 = any & ~flip;
    uint32_t acc = flip, tied = ~flip;
    const uint32_t urow = __builtin_amdgcn_readfirstlane(row);
    const Words4 b0 = philox4x32_10<2, 3>(g, urow, t, (uint32_t)Q, key0, key1);
    const Words4 b1 = philox4x32_10<2, 3>(g, urow, t, 2u + (uint32_t)Q, key0, key1);
    compare_planes(acc, tied, sel2, b0, th, 0u);
    compare_planes(acc, tied, sel2, b1, th, 1u);
    if (O) own.o ^= acc; else own.e ^= acc;
    const uint64_t B = __builtin_amdgcn_ballot_w64(tied != 0u);
    const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(B >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)B, 0u));
    const uint32_t pos = tied != 0u ? n + rank : kPairQueueCap + lane;
    q.task[pos] = make_uint4(tied, sel2 & tied, urow, (uint32_t)U | (lane << 3) | (g << 9));
    n += (uint32_t)__builtin_popcountll(B);
}

// Settles the n queued words, one per lane, with the planes of blocks 2 onwards.  Update u of the pair
// (u & 3 = white t, black t, white t + 1, black t + 1) has sweep t + ((u >> 1) & 1) and colour 1 - (u & 1).
__device__ __forceinline__ void pair_settle(const PairQueue& q, uint32_t n, const Thresholds& th, uint32_t t,
                                            uint32_t key0, uint32_t key1, uint32_t lane) {
    wave_lds_sync();
#pragma unroll 1
    for (uint32_t b = 0; b < n; b += 64u) {
        const uint32_t j = b + lane;
        const bool have = j < n;
        uint4 e = make_uint4(0u, 0u, 0u, 0u);
        if (have) e = q.task[j];
        uint32_t tied = e.x;
        const uint32_t s2 = e.y, row = e.z, meta = e.w;
        const uint32_t u = meta & 7u, src = (meta >> 3) & 63u, g = meta >> 9;
        const uint32_t tu = t + ((u >> 1) & 1u), qu = (u & 1u) ^ 1u;
        uint32_t acc = 0u;
        // blocks 2 and 3 as two independent chains (a queue of a few dozen words almost always needs both;
        // a block that finds no tied site changes nothing), then one at a time
        if (wave_any(tied != 0u)) {
            const Words4 b2 = philox4x32_10(g, row, tu, 4u + qu, key0, key1);
            const Words4 b3 = philox4x32_10(g, row, tu, 6u + qu, key0, key1);
            compare_planes(acc, tied, s2, b2, th, 2u);
            compare_planes(acc, tied, s2, b3, th, 3u);
        }
#pragma unroll 1
        for (uint32_t m = 4; m < th.blocks; ++m) {
            if (!wave_any(tied != 0u)) break;
            compare_planes(acc, tied, s2, philox4x32_10(g, row, tu, 2u * m + qu, key0, key1), th, m);
        }
        if (have) q.res[64u * u + src] = acc;
    }
    wave_lds_sync();
}

// The strip holds rows r0 .. r0 + R - 1 (pair_strip_rows).
template <bool OBS, bool STAGED, bool UP>
__device__ __forceinline__ void fused2p_strip(const FusedArgs& a, uint32_t r0_, uint32_t R, uint4* fused_lds,
                                              Counts& ct, Counts& ct1) {
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    const uint32_t G = a.groups, L = a.L;
    uint32_t* const wl = reinterpret_cast<uint32_t*>(fused_lds) + (tid >> 6) * (kPairWaveBytes / 4u);
    uint4* const stage = reinterpret_cast<uint4*>(wl);
    uint32_t* const xch = reinterpret_cast<uint32_t*>(fused_lds) + (nt >> 6) * (kPairWaveBytes / 4u);
    const PairQueue q{reinterpret_cast<uint4*>(wl), wl + 4u * kPairQueueSlots};
    const bool active = tid < G;
    const uint32_t g = active ? tid : G - 1;
    const uint32_t gl = g == 0 ? G - 1 : g - 1, gr = g + 1 == G ? 0 : g + 1;
    const uint32_t lane = tid & 63u;
    const uint32_t r0 = __builtin_amdgcn_readfirstlane(r0_);  // uniform: keeps the row arithmetic scalar
    const size_t col = (size_t)(STAGED ? g - lane : g) * 64u;
    // walk row k = 0 .. R + 7: r0 - 4 .. r0 + R + 3 (down) or r0 + R + 3 .. r0 - 4 (up), wrapped onto the
    // torus; callers pass k <= R + 7 for every row they load or store
    auto vrow = [&](uint32_t k) {
        const int32_t v = (int32_t)(UP ? r0 + R + 3 - k : r0 + k) - (UP ? 0 : 4);  // in [-4, L + 4)
        return (uint32_t)(v < 0 ? v + (int32_t)L : v >= (int32_t)L ? v - (int32_t)L : v);
    };
    auto fetch = [&](Row& raw, uint32_t r) {
        if (STAGED) load_row_coalesced(raw, a.src + (size_t)r * L + col, lane);
        else load_row(raw, a.src + (size_t)r * L + col);
    };
    auto own = [&](const Row& raw) {
        if (!STAGED) return row_bits(raw);
        Row row;
        regroup_to_owner(row, raw, stage, lane);
        return row_bits(row);
    };
    auto put = [&](uint32_t r, const RowBits& b) {
        Row row;
        bits_to_row(row, b);
        if (STAGED) store_row_coalesced(a.dst + (size_t)r * L + col, row, stage, lane, a.nt_store);
        else if (active) store_row(a.dst + (size_t)r * L + col, row, a.nt_store);
    };
    // Window at the start of the pair of steps s, s + 1 (s even): w_j = walk row s + 3 - j, j = 0 .. 12.
    // The updates of step s lie on columns of parity OA, those of step s + 1 on OB.
    constexpr int OA = UP ? 1 : 0, OB = 1 - OA;
    const uint32_t t = a.t, k0 = a.key0, k1 = a.key1;
    const RowBits z{0u, 0u};
    RowBits w12 = z, w11 = z, w10 = z, w9 = z, w8 = z, w7 = z, w6 = z, w5 = z, w4 = z;
    Row rawA, rawB;
    fetch(rawA, vrow(0));
    RowBits w3 = own(rawA);
    fetch(rawA, vrow(1));
    RowBits w2 = own(rawA);
    fetch(rawA, vrow(2));
    RowBits w1 = own(rawA);
    fetch(rawA, vrow(3));
    RowBits w0 = own(rawA);
    fetch(rawA, vrow(4));
    fetch(rawB, vrow(5));
    xch[tid] = pair_edges(w2, w5, w8, w11, w1, w4, w7, w10);
    workgroup_lds_sync();
#pragma unroll 1
    for (uint32_t s = 0; s < R + 12; s += 2) {
        // a wave's issue priority falls as it walks (3 in the first quarter of its pairs, 0 in the last).
        // The instruction arbiter otherwise favours the oldest wave, so the workgroups dispatched last ran
        // almost twice as long as the first ones and each SIMD ended with one wave alone.
        switch ((4u * s) / (R + 12u)) {
            case 0: __builtin_amdgcn_s_setprio(3); break;
            case 1: __builtin_amdgcn_s_setprio(2); break;
            case 2: __builtin_amdgcn_s_setprio(1); break;
            default: __builtin_amdgcn_s_setprio(0); break;
        }
        const uint32_t sl = ((s >> 1) & 1u) * nt;
        const uint32_t nbL = xch[sl + gl], nbR = xch[sl + gr];
        // step s makes U1 for s <= R + 5, U2 for 4 <= s <= R + 7, U3 for 8 <= s <= R + 9, U4 for 12 <= s
        const uint32_t s1 = s + 1u;
        const bool u1a = s <= R + 5, u1b = s1 <= R + 5;
        const bool u2a = s >= 4u && s <= R + 7, u2b = s1 >= 4u && s1 <= R + 7;
        const bool u3a = s >= 8u && s <= R + 9, u3b = s1 >= 8u && s1 <= R + 9;
        const bool u4a = s >= 12u, u4b = s1 >= 12u;
#pragma unroll
        for (uint32_t u = 0; u < 8u; ++u) q.res[64u * u + lane] = 0u;
        uint32_t n = 0u;
        if (u1a) pair_update<OA, 1, 0>(w2, w3, w1, nbL, nbR, a.th, g, vrow(s + 1u), t, k0, k1, q, n, lane);
        if (u2a) pair_update<OA, 0, 1>(w5, w6, w4, nbL, nbR, a.th, g, vrow(s - 2u), t, k0, k1, q, n, lane);
        if (u3a) pair_update<OA, 1, 2>(w8, w9, w7, nbL, nbR, a.th, g, vrow(s - 5u), t + 1u, k0, k1, q, n, lane);
        if (u4a) pair_update<OA, 0, 3>(w11, w12, w10, nbL, nbR, a.th, g, vrow(s - 8u), t + 1u, k0, k1, q, n, lane);
        if (u1b) pair_update<OB, 1, 4>(w1, w2, w0, nbL, nbR, a.th, g, vrow(s + 2u), t, k0, k1, q, n, lane);
        if (u2b) pair_update<OB, 0, 5>(w4, w5, w3, nbL, nbR, a.th, g, vrow(s - 1u), t, k0, k1, q, n, lane);
        if (u3b) pair_update<OB, 1, 6>(w7, w8, w6, nbL, nbR, a.th, g, vrow(s - 4u), t + 1u, k0, k1, q, n, lane);
        if (u4b) pair_update<OB, 0, 7>(w10, w11, w9, nbL, nbR, a.th, g, vrow(s - 7u), t + 1u, k0, k1, q, n, lane);
        pair_settle(q, n, a.th, t, k0, k1, lane);
        // zero for the updates the pair does not make
        const uint4 ra = make_uint4(q.res[lane], q.res[64u + lane], q.res[128u + lane], q.res[192u + lane]);
        const uint4 rb = make_uint4(q.res[256u + lane], q.res[320u + lane], q.res[384u + lane], q.res[448u + lane]);
        if (OA) { w2.o ^= ra.x; w5.o ^= ra.y; w8.o ^= ra.z; w11.o ^= ra.w; w1.e ^= rb.x; w4.e ^= rb.y; w7.e ^= rb.z; w10.e ^= rb.w; }
        else { w2.e ^= ra.x; w5.e ^= ra.y; w8.e ^= ra.z; w11.e ^= ra.w; w1.o ^= rb.x; w4.o ^= rb.y; w7.o ^= rb.z; w10.o ^= rb.w; }
        if (OBS) {
            // sweep t: the black update of an own row (walk rows 4 .. R + 3); sweep t + 1: every U4 row
            if (s >= 6u && s <= R + 5) tq_count<OA, 1>(w5, w6, w4, nbL, nbR, ct);
            if (s1 >= 6u && s1 <= R + 5) tq_count<OB, 5>(w4, w5, w3, nbL, nbR, ct);
            if (u4a) tq_count<OA, 3>(w11, w12, w10, nbL, nbR, ct1);
            if (u4b) tq_count<OB, 7>(w10, w11, w9, nbL, nbR, ct1);
        }
        // walk rows s + 4, s + 5 (fetched a pair ago), the rows the pair finished, and the requests for
        // s + 6, s + 7 (past the walk's last row the last row again; those rows are never updated).  The
        // vector-memory counter also counts stores: converting the fetched rows before the stores keeps
        // their waits from draining the stores just issued.
        const RowBits n4 = own(rawA), n5 = own(rawB);
        if (u4a) put(vrow(s - 8u), w11);
        if (u4b) put(vrow(s - 7u), w10);
        fetch(rawA, vrow(s + 6u <= R + 7 ? s + 6u : R + 7));
        fetch(rawB, vrow(s + 7u <= R + 7 ? s + 7u : R + 7));
        w12 = w10; w11 = w9; w10 = w8; w9 = w7; w8 = w6; w7 = w5; w6 = w4; w5 = w3; w4 = w2; w3 = w1; w2 = w0;
        w1 = n4;
        w0 = n5;
        xch[(((s >> 1) + 1u) & 1u) * nt + tid] = pair_edges(w2, w5, w8, w11, w1, w4, w7, w10);
        workgroup_lds_sync();
    }
}

template <bool OBS, bool STAGED>
__global__ __launch_bounds__(512) void k_sweep_fused2p(FusedArgs a) {
    extern __shared__ uint4 fused_lds[];
    const uint32_t strip = logical_block(blockIdx.x, gridDim.x, a.xcd_remap);
    uint32_t R;
    const uint32_t r0 = pair_strip_rows(strip, gridDim.x, a.rows, a.tall, R);
    Counts ct{0u, 0u}, ct1{0u, 0u};
    if (a.alternate && (strip & 1u)) fused2p_strip<OBS, STAGED, true>(a, r0, R, fused_lds, ct, ct1);
    else fused2p_strip<OBS, STAGED, false>(a, r0, R, fused_lds, ct, ct1);
    const bool active = threadIdx.x < a.groups;
    if (OBS) {
        int64_t* const out = a.spread ? spread_line(a.obs, blockIdx.x) : a.obs;
        block_accumulate(out, active ? ct.anti : 0u, active ? ct.neg : 0u, active ? 1u : 0u, 64u * R);
        __syncthreads();  // block_accumulate's LDS is reused
        block_accumulate(out + 2, active ? ct1.anti : 0u, active ? ct1.neg : 0u, active ? 1u : 0u, 64u * R);
    }
}

// ---- Two sweeps per pass in column bands of one wave.
//
// The pass above puts a whole row in one workgroup, one thread per 64-column group, so it stops at
// L = 65536.  Here (L >= 4096) a band of one wave walks a strip of R rows instead, over 64 consecutive groups
// (modulo the row) of which the middle ones are its own: lane l takes group b0 - 1 + l, lanes
// 1 .. n of them (n <= 62) are the band's groups, and lane 0 and the lanes past n only recompute their
// groups so that the band's own sites see correct neighbours.  The group-edge neighbours come from the
// adjacent lanes by a lane shift (no LDS exchange, no workgroup barrier: every wave is independent).
// The shift brings nothing into lane 0 from the left or into lane 63 from the right; a wrong value at
// a band's edge spreads by at most one column per colour update, four columns over the pass, so it
// never reaches the neighbour group of an own one (the light cone of Sec. 3.1's colour updates).  Rows
// are recomputed four deep above and below the strip as in the full-row pass.  The walk, the
// uniforms and the tie queue are those of the full-row pass, so the result is the same two sweeps,
// bit for bit.
struct BandArgs {
    const int8_t* src;
    int8_t* dst;
    uint32_t L, groups, rows;  // rows = R, even, divides L
    uint32_t bands;            // bands per row; band b owns groups [b G / bands, (b + 1) G / bands)
    uint32_t units;            // bands x strips
    uint32_t t, key0, key1;
    Thresholds th;
    int64_t* obs;        // OBS: (M, E) after sweep t, then after t + 1, zeroed beforehand
    uint32_t xcd_remap;  // renumber blocks per XCD (see logical_block)
    uint32_t nt_store;   // non-temporal stores of the output rows
    uint32_t alternate;  // walk odd strips upwards
};

// lane l's value of v from lane l - 1 (to the left; lane 0 gets 0) and from lane l + 1 (lane 63 gets 0)
__device__ __forceinline__ uint32_t from_left_lane(uint32_t v) {
    return __builtin_amdgcn_update_dpp(0u, v, 0x138, 0xF, 0xF, false);  // wave_shr:1
}
__device__ __forceinline__ uint32_t from_right_lane(uint32_t v) {
    return __builtin_amdgcn_update_dpp(0u, v, 0x130, 0xF, 0xF, false);  // wave_shl:1
}

// Band b's first own group and its number of own groups (at most 62; uniform).
__device__ __forceinline__ uint32_t band_first(const BandArgs& a, uint32_t band) {
    return (uint32_t)((uint64_t)band * a.groups / a.bands);
}
__device__ __forceinline__ uint32_t band_width(const BandArgs& a, uint32_t band) {
    return (uint32_t)((uint64_t)(band + 1) * a.groups / a.bands) - band_first(a, band);
}

template <bool OBS, bool UP>
__device__ __forceinline__ void fused2b_strip(const BandArgs& a, uint32_t band, uint32_t strip, uint4* stage,
                                              uint32_t lane, Counts& ct, Counts& ct1) {
    const uint32_t G = a.groups, L = a.L, R = a.rows;
    const TieQueue q{reinterpret_cast<uint32_t*>(stage), stage + 256};
    const uint32_t b0 = band_first(a, band), n_own = band_width(a, band);
    // b0 + G - 1 + lane < 3G since G >= 64
    uint32_t g = b0 + G - 1u + lane;
    g = g >= G ? g - G : g;
    g = g >= G ? g - G : g;
    // the row group of the band group lane / 4 (the lane's coalesced chunks are in band groups
    // lane / 4 + 16 k; those in band groups 1 .. n_own are stored)
    uint32_t gbase = b0 + G - 1u + (lane >> 2);
    gbase = gbase >= G ? gbase - G : gbase;
    gbase = gbase >= G ? gbase - G : gbase;
    const uint32_t r0 = __builtin_amdgcn_readfirstlane(strip * R);  // uniform: keeps the row arithmetic scalar
    auto vrow = [&](uint32_t k) {
        const uint32_t kk = k < R + 7 ? k : R + 7;
        // in [-4, L + 4) since r0 + R <= L; signed compares keep the wrap on the scalar unit
        const int32_t v = (int32_t)(UP ? r0 + R + 3 - kk : r0 + kk) - (UP ? 0 : 4);
        return (uint32_t)(v < 0 ? v + (int32_t)L : v >= (int32_t)L ? v - (int32_t)L : v);
    };
    auto fetch = [&](Row& raw, uint32_t r) { load_row_chunks(raw, a.src + (size_t)r * L, gbase, G, lane); };
    auto own = [&](const Row& raw) {
        Row row;
        regroup_to_owner(row, raw, stage, lane);
        return row_bits(row);
    };
    auto put = [&](uint32_t r, const RowBits& b) {
        Row row;
        bits_to_row(row, b);
        store_row_chunks(a.dst + (size_t)r * L, row, stage, lane, gbase, G, n_own, a.nt_store);
    };
    constexpr int OA = UP ? 1 : 0, OB = 1 - OA;
    const uint32_t t = a.t, k0 = a.key0, k1 = a.key1;
    Row raw;
    fetch(raw, vrow(0));
    RowBits w7{0u, 0u}, w6{0u, 0u}, w5{0u, 0u}, w4{0u, 0u}, w3{0u, 0u}, w2{0u, 0u};
    RowBits w1 = own(raw);
    fetch(raw, vrow(1));
    RowBits w0 = own(raw);
    fetch(raw, vrow(2));
    RowBits nx = own(raw);
    fetch(raw, vrow(3));
    uint32_t e = edge_word4(w0, w2, w4, w6);
#define ISING_FUSED2B_STEP(O, S)                                                                             \
    do {                                                                                                     \
        const uint32_t s_ = (S);                                                                             \
        const uint32_t act = (s_ <= R + 5 ? 1u : 0u) | (s_ >= 3 && s_ <= R + 6 ? 2u : 0u) |                 \
                             (s_ >= 6 && s_ <= R + 7 ? 4u : 0u) | (s_ >= 9 && s_ <= R + 8 ? 8u : 0u);        \
        const uint32_t rw[4] = {vrow(s_ + 1), s_ >= 1 ? vrow(s_ - 1) : 0u, s_ >= 3 ? vrow(s_ - 3) : 0u,      \
                                s_ >= 5 ? vrow(s_ - 5) : 0u};                                                \
        fused2q_step<O, OBS>(w0, w2, w4, w6, nx, w1, w3, w5, w7, from_left_lane(e), from_right_lane(e), a.th,  \
                             g, rw, act, t, k0, k1, q, lane, ct, ct1, s_ >= 5 && s_ <= R + 4);                \
        if (act & 8u) put(rw[3], w6);                                                                        \
        w7 = w6; w6 = w5; w5 = w4; w4 = w3; w3 = w2; w2 = w1; w1 = w0; w0 = nx;                              \
        e = edge_word4(w0, w2, w4, w6);                                                                      \
        nx = own(raw);  /* walk row s + 3 */                                                                 \
        fetch(raw, vrow(s_ + 4));                                                                            \
    } while (0)
#pragma unroll 1
    for (uint32_t s = 0; s < R + 10; s += 2) {  // step R + 9 makes no update
        ISING_FUSED2B_STEP(OA, s);
        ISING_FUSED2B_STEP(OB, s + 1);
    }
#undef ISING_FUSED2B_STEP
}

// One wave per (band, strip) unit; units are numbered band-fastest within a strip, and the XCD
// renumbering hands each XCD a contiguous range of them (vertically adjacent strips share rows).
template <bool OBS>
__global__ __launch_bounds__(256, 4) void k_sweep_fused2b(BandArgs a) {
    extern __shared__ uint4 band_lds[];
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint32_t unit = logical_block(blockIdx.x, gridDim.x, a.xcd_remap) * (blockDim.x >> 6) + wave;
    uint4* const stage = band_lds + wave * (kTieQueueBytes / 16u);
    Counts ct{0u, 0u}, ct1{0u, 0u};
    const bool live = unit < a.units;  // uniform per wave
    const uint32_t band = live ? unit % a.bands : 0u, strip = live ? unit / a.bands : 0u;
    if (live) {
        if (a.alternate && (strip & 1u)) fused2b_strip<OBS, true>(a, band, strip, stage, lane, ct, ct1);
        else fused2b_strip<OBS, false>(a, band, strip, stage, lane, ct, ct1);
    }
    if (OBS) {
        const bool own = live && lane >= 1u && lane <= band_width(a, band);
        block_accumulate(a.obs, own ? ct.anti : 0u, own ? ct.neg : 0u, own ? 1u : 0u, 64u * a.rows);
        __syncthreads();  // block_accumulate's LDS is reused
        block_accumulate(a.obs + 2, own ? ct1.anti : 0u, own ? ct1.neg : 0u, own ? 1u : 0u, 64u * a.rows);
    }
}

// ---- The paired two-sweep walk (k_sweep_fused2p) in column bands of one wave (k_sweep_fused2b): the band's
// lanes, its recomputed edge groups and its row I/O are those of the band pass, the walk, the uniforms and
// the tie queue those of the paired pass; the group-edge words come from the adjacent lanes by lane shifts,
// once per pair.  A wrong value at a band's edge still spreads by at most four columns over the pass (four
// colour updates), so the result is the same two sweeps, bit for bit.
template <bool OBS, bool UP>
__device__ __forceinline__ void fused2pb_strip(const BandArgs& a, uint32_t band, uint32_t strip, uint32_t* wl,
                                               uint32_t lane, Counts& ct, Counts& ct1) {
    const uint32_t G = a.groups, L = a.L, R = a.rows;
    uint4* const stage = reinterpret_cast<uint4*>(wl);
    const PairQueue q{reinterpret_cast<uint4*>(wl), wl + 4u * kPairQueueSlots};
    const uint32_t b0 = band_first(a, band), n_own = band_width(a, band);
    // b0 + G - 1 + lane < 3G since G >= 64
    uint32_t g = b0 + G - 1u + lane;
    g = g >= G ? g - G : g;
    g = g >= G ? g - G : g;
    uint32_t gbase = b0 + G - 1u + (lane >> 2);
    gbase = gbase >= G ? gbase - G : gbase;
    gbase = gbase >= G ? gbase - G : gbase;
    const uint32_t r0 = __builtin_amdgcn_readfirstlane(strip * R);  // uniform: keeps the row arithmetic scalar
    auto vrow = [&](uint32_t k) {
        const int32_t v = (int32_t)(UP ? r0 + R + 3 - k : r0 + k) - (UP ? 0 : 4);  // in [-4, L + 4)
        return (uint32_t)(v < 0 ? v + (int32_t)L : v >= (int32_t)L ? v - (int32_t)L : v);
    };
    auto fetch = [&](Row& raw, uint32_t r) { load_row_chunks(raw, a.src + (size_t)r * L, gbase, G, lane); };
    auto own = [&](const Row& raw) {
        Row row;
        regroup_to_owner(row, raw, stage, lane);
        return row_bits(row);
    };
    auto put = [&](uint32_t r, const RowBits& b) {
        Row row;
        bits_to_row(row, b);
        store_row_chunks(a.dst + (size_t)r * L, row, stage, lane, gbase, G, n_own, a.nt_store);
    };
    constexpr int OA = UP ? 1 : 0, OB = 1 - OA;
    const uint32_t t = a.t, k0 = a.key0, k1 = a.key1;
    const RowBits z{0u, 0u};
    RowBits w12 = z, w11 = z, w10 = z, w9 = z, w8 = z, w7 = z, w6 = z, w5 = z, w4 = z;
    Row rawA, rawB;
    fetch(rawA, vrow(0));
    RowBits w3 = own(rawA);
    fetch(rawA, vrow(1));
    RowBits w2 = own(rawA);
    fetch(rawA, vrow(2));
    RowBits w1 = own(rawA);
    fetch(rawA, vrow(3));
    RowBits w0 = own(rawA);
    fetch(rawA, vrow(4));
    fetch(rawB, vrow(5));
    uint32_t e = pair_edges(w2, w5, w8, w11, w1, w4, w7, w10);
#pragma unroll 1
    for (uint32_t s = 0; s < R + 12; s += 2) {
        switch ((4u * s) / (R + 12u)) {  // issue priority falling along the walk (as in k_sweep_fused2p)
            case 0: __builtin_amdgcn_s_setprio(3); break;
            case 1: __builtin_amdgcn_s_setprio(2); break;
            case 2: __builtin_amdgcn_s_setprio(1); break;
            default: __builtin_amdgcn_s_setprio(0); break;
        }
        const uint32_t nbL = from_left_lane(e), nbR = from_right_lane(e);
        const uint32_t s1 = s + 1u;
        const bool u1a = s <= R + 5, u1b = s1 <= R + 5;
        const bool u2a = s >= 4u && s <= R + 7, u2b = s1 >= 4u && s1 <= R + 7;
        const bool u3a = s >= 8u && s <= R + 9, u3b = s1 >= 8u && s1 <= R + 9;
        const bool u4a = s >= 12u, u4b = s1 >= 12u;
#pragma unroll
        for (uint32_t u = 0; u < 8u; ++u) q.res[64u * u + lane] = 0u;
        uint32_t n = 0u;
        if (u1a) pair_update<OA, 1, 0>(w2, w3, w1, nbL, nbR, a.th, g, vrow(s + 1u), t, k0, k1, q, n, lane);
        if (u2a) pair_update<OA, 0, 1>(w5, w6, w4, nbL, nbR, a.th, g, vrow(s - 2u), t, k0, k1, q, n, lane);
        if (u3a) pair_update<OA, 1, 2>(w8, w9, w7, nbL, nbR, a.th, g, vrow(s - 5u), t + 1u, k0, k1, q, n, lane);
        if (u4a) pair_update<OA, 0, 3>(w11, w12, w10, nbL, nbR, a.th, g, vrow(s - 8u), t + 1u, k0, k1, q, n, lane);
        if (u1b) pair_update<OB, 1, 4>(w1, w2, w0, nbL, nbR, a.th, g, vrow(s + 2u), t, k0, k1, q, n, lane);
        if (u2b) pair_update<OB, 0, 5>(w4, w5, w3, nbL, nbR, a.th, g, vrow(s - 1u), t, k0, k1, q, n, lane);
        if (u3b) pair_update<OB, 1, 6>(w7, w8, w6, nbL, nbR, a.th, g, vrow(s - 4u), t + 1u, k0, k1, q, n, lane);
        if (u4b) pair_update<OB, 0, 7>(w10, w11, w9, nbL, nbR, a.th, g, vrow(s - 7u), t + 1u, k0, k1, q, n, lane);
        pair_settle(q, n, a.th, t, k0, k1, lane);
        const uint4 ra = make_uint4(q.res[lane], q.res[64u + lane], q.res[128u + lane], q.res[192u + lane]);
        const uint4 rb = make_uint4(q.res[256u + lane], q.res[320u + lane], q.res[384u + lane], q.res[448u + lane]);
        if (OA) { w2.o ^= ra.x; w5.o ^= ra.y; w8.o ^= ra.z; w11.o ^= ra.w; w1.e ^= rb.x; w4.e ^= rb.y; w7.e ^= rb.z; w10.e ^= rb.w; }
        else { w2.e ^= ra.x; w5.e ^= ra.y; w8.e ^= ra.z; w11.e ^= ra.w; w1.o ^= rb.x; w4.o ^= rb.y; w7.o ^= rb.z; w10.o ^= rb.w; }
        if (OBS) {
            if (s >= 6u && s <= R + 5) tq_count<OA, 1>(w5, w6, w4, nbL, nbR, ct);
            if (s1 >= 6u && s1 <= R + 5) tq_count<OB, 5>(w4, w5, w3, nbL, nbR, ct);
            if (u4a) tq_count<OA, 3>(w11, w12, w10, nbL, nbR, ct1);
            if (u4b) tq_count<OB, 7>(w10, w11, w9, nbL, nbR, ct1);
        }
        const RowBits n4 = own(rawA), n5 = own(rawB);
        if (u4a) put(vrow(s - 8u), w11);
        if (u4b) put(vrow(s - 7u), w10);
        fetch(rawA, vrow(s + 6u <= R + 7 ? s + 6u : R + 7));
        fetch(rawB, vrow(s + 7u <= R + 7 ? s + 7u : R + 7));
        w12 = w10; w11 = w9; w10 = w8; w9 = w7; w8 = w6; w7 = w5; w6 = w4; w5 = w3; w4 = w2; w3 = w1; w2 = w0;
        w1 = n4;
        w0 = n5;
        e = pair_edges(w2, w5, w8, w11, w1, w4, w7, w10);
    }
}

// One wave per (band, strip) unit, numbered as for k_sweep_fused2b; up to 168 registers, three waves per
// SIMD.
template <bool OBS>
__global__ __launch_bounds__(256, 3) void k_sweep_fused2pb(BandArgs a) {
    extern __shared__ uint4 band_lds[];
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint32_t unit = logical_block(blockIdx.x, gridDim.x, a.xcd_remap) * (blockDim.x >> 6) + wave;
    uint32_t* const wl = reinterpret_cast<uint32_t*>(band_lds) + wave * (kPairWaveBytes / 4u);
    Counts ct{0u, 0u}, ct1{0u, 0u};
    const bool live = unit < a.units;  // uniform per wave
    const uint32_t band = live ? unit % a.bands : 0u, strip = live ? unit / a.bands : 0u;
    if (live) {
        if (a.alternate && (strip & 1u)) fused2pb_strip<OBS, true>(a, band, strip, wl, lane, ct, ct1);
        else fused2pb_strip<OBS, false>(a, band, strip, wl, lane, ct, ct1);
    }
    if (OBS) {
        const bool own = live && lane >= 1u && lane <= band_width(a, band);
        block_accumulate(a.obs, own ? ct.anti : 0u, own ? ct.neg : 0u, own ? 1u : 0u, 64u * a.rows);
        __syncthreads();  // block_accumulate's LDS is reused
        block_accumulate(a.obs + 2, own ? ct1.anti : 0u, own ? ct1.neg : 0u, own ? 1u : 0u, 64u * a.rows);
    }
}

// ---- One sweep per pass with the ties of a step settled together: the one-sweep walk with two
// rows between its updates.  Step s updates the white sites of walk row s + 1 and the black sites
// of walk row s - 1; neither reads what the other writes, so the two are independent and share
// the tie queue (as in the two-sweep pass).  Same rows read and written as k_sweep_fused, same
// uniforms, same result.
template <bool OBS, bool STAGED, bool UP>
__device__ __forceinline__ void fusedq_strip(const FusedArgs& a, uint32_t strip, uint4* fused_lds, Counts& ct) {
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    const uint32_t G = a.groups, L = a.L, R = a.rows;
    uint4* const stage = fused_lds + (tid >> 6) * (kTieQueueBytes / 16u);
    uint32_t* const xch = reinterpret_cast<uint32_t*>(fused_lds + (nt >> 6) * (kTieQueueBytes / 16u));
    const TieQueue q{reinterpret_cast<uint32_t*>(stage), stage + 256};
    const bool active = tid < G;
    const uint32_t g = active ? tid : G - 1;
    const uint32_t gl = g == 0 ? G - 1 : g - 1, gr = g + 1 == G ? 0 : g + 1;
    const uint32_t lane = tid & 63u;
    const uint32_t r0 = __builtin_amdgcn_readfirstlane(strip * R);  // uniform: keeps the row arithmetic scalar
    const size_t col = (size_t)(STAGED ? g - lane : g) * 64u;
    // walk row k = 0 .. R + 3: r0 - 2 .. r0 + R + 1 (down) or r0 + R + 1 .. r0 - 2 (up), wrapped;
    // prefetches past the last walk row are clamped to it
    auto vrow = [&](uint32_t k) {
        const uint32_t kk = k < R + 3 ? k : R + 3;
        const uint32_t v = UP ? r0 + R + 1 + L - kk : r0 + L + kk - 2;  // in [L - 2, 2L + 2)
        return v >= 2 * L ? v - 2 * L : v >= L ? v - L : v;
    };
    auto fetch = [&](Row& raw, uint32_t r) {
        if (STAGED) load_row_coalesced(raw, a.src + (size_t)r * L + col, lane);
        else load_row(raw, a.src + (size_t)r * L + col);
    };
    auto own = [&](const Row& raw) {
        if (!STAGED) return row_bits(raw);
        Row row;
        regroup_to_owner(row, raw, stage, lane);
        return row_bits(row);
    };
    auto put = [&](uint32_t r, const RowBits& b) {
        Row row;
        bits_to_row(row, b);
        if (STAGED) store_row_coalesced(a.dst + (size_t)r * L + col, row, stage, lane, a.nt_store);
        else if (active) store_row(a.dst + (size_t)r * L + col, row, a.nt_store);
    };
    // Step s makes the white update for s <= R + 1 (walk rows 1 .. R + 2) and the black one for
    // 3 <= s <= R + 2 (walk rows 2 .. R + 1, the strip's own rows, written after their update).
    // The white update of an even step lies on columns of parity OA, the black one on 1 - OA.
    constexpr int OA = UP ? 1 : 0, OB = 1 - OA;
    const uint32_t t = a.t, k0 = a.key0, k1 = a.key1;
    Row raw;
    fetch(raw, vrow(0));
    RowBits w3{0u, 0u}, w2{0u, 0u};
    RowBits w1 = own(raw);
    fetch(raw, vrow(1));
    RowBits w0 = own(raw);
    fetch(raw, vrow(2));
    RowBits nx = own(raw);
    fetch(raw, vrow(3));
    xch[tid] = edge_word4(w0, w2, w0, w0);  // slot 0: walk row 1 (pair 0), pair 1 unused yet
    workgroup_lds_sync();
#define ISING_FUSEDQ_STEP(O, S)                                                                              \
    do {                                                                                                     \
        constexpr int X_ = 1 - (O);                                                                          \
        const uint32_t s_ = (S);                                                                             \
        const bool a1 = s_ <= R + 1, a2 = s_ >= 3 && s_ <= R + 2;                                            \
        const uint32_t sl = (s_ & 1u) * nt;                                                                  \
        const uint32_t nbL = xch[sl + gl], nbR = xch[sl + gr];                                               \
        const uint32_t rw1 = vrow(s_ + 1), rw2 = s_ >= 1 ? vrow(s_ - 1) : 0u;                                \
        q.res[lane] = make_uint4(0u, 0u, 0u, 0u);                                                            \
        uint32_t n = 0u;                                                                                     \
        if (a1) tq_update<(O), 1, 0>(w0, nx, w1, nbL, nbR, a.th, g, rw1, t, k0, k1, q, n, lane);             \
        if (a2) tq_update<X_, 0, 1>(w2, w1, w3, nbL, nbR, a.th, g, rw2, t, k0, k1, q, n, lane);              \
        tq_settle<-1>(q, n, a.th, t, k0, k1, lane);                                                          \
        const uint4 r_ = q.res[lane];                                                                        \
        if (O) { w0.o ^= r_.x; w2.e ^= r_.y; } else { w0.e ^= r_.x; w2.o ^= r_.y; }                          \
        if (a2) {                                                                                            \
            if (OBS) tq_count<X_, 1>(w2, w1, w3, nbL, nbR, ct);                                              \
            put(rw2, w2);                                                                                    \
        }                                                                                                    \
        w3 = w2; w2 = w1; w1 = w0; w0 = nx;                                                                  \
        xch[((s_ + 1) & 1u) * nt + tid] = edge_word4(w0, w2, w0, w0);                                        \
        nx = own(raw); /* walk row s + 3 */                                                                  \
        fetch(raw, vrow(s_ + 4));                                                                            \
        workgroup_lds_sync();                                                                                \
    } while (0)
#pragma unroll 1
    for (uint32_t s = 0; s < R + 4; s += 2) {  // step R + 3 makes no update
        ISING_FUSEDQ_STEP(OA, s);
        ISING_FUSEDQ_STEP(OB, s + 1);
    }
#undef ISING_FUSEDQ_STEP
}

template <bool OBS, bool STAGED>
__global__ __launch_bounds__(1024) void k_sweep_fusedq(FusedArgs a) {
    extern __shared__ uint4 fused_lds[];
    const uint32_t strip = logical_block(blockIdx.x, gridDim.x, a.xcd_remap);
    Counts ct{0u, 0u};
    if (a.alternate && (strip & 1u)) fusedq_strip<OBS, STAGED, true>(a, strip, fused_lds, ct);
    else fusedq_strip<OBS, STAGED, false>(a, strip, fused_lds, ct);
    const bool active = threadIdx.x < a.groups;
    if (OBS) block_accumulate(a.obs, active ? ct.anti : 0u, active ? ct.neg : 0u, active ? 1u : 0u, 64u * a.rows);
}

// ---- observables of an int8 lattice: M = sum of spins, E = -sum over bonds (right, down).
struct ObsArgs {
    const int8_t* spins;
    uint32_t L, groups, rows, n_lanes;
    int64_t* out;
};

__global__ __launch_bounds__(256) void k_observables_int8(ObsArgs a) {
    const uint32_t lane_id = blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = lane_id < a.n_lanes;
    uint32_t anti = 0, neg = 0, units = 0;
    if (active) {
        const uint32_t g = lane_id % a.groups;
        const uint32_t strip = lane_id / a.groups;
        const uint32_t L = a.L;
        const uint32_t gr = g + 1 == a.groups ? 0 : g + 1;
        // a half group (the last 32 columns of a row whose length is an odd multiple of 32) has 8
        // dwords; its right neighbour is column 0 of the row
        const bool half = (L & 63u) != 0 && gr == 0;
        const uint32_t nd = half ? 8u : 16u;
        units = half ? 1u : 2u;
        const int8_t* col = a.spins + (size_t)g * 64u;
        Row cur, dn;
        uint32_t r = strip * a.rows;
        if (half) load_row_half(cur, col + (size_t)r * L);
        else load_row(cur, col + (size_t)r * L);
#pragma unroll 1
        for (uint32_t s = 0; s < a.rows; ++s, ++r) {
            const uint32_t rd = r + 1 == L ? 0 : r + 1;
            if (half) load_row_half(dn, col + (size_t)rd * L);
            else load_row(dn, col + (size_t)rd * L);
            const uint32_t right = *reinterpret_cast<const uint32_t*>(a.spins + (size_t)r * L + (size_t)gr * 64u);
#pragma unroll
            for (uint32_t k = 0; k < 16; ++k) {
                if (k < nd) {
                    const uint32_t nb = k + 1 < nd ? cur.d[(k + 1) & 15u] : right;
                    const uint32_t rn = __builtin_amdgcn_alignbyte(nb, cur.d[k], 1);  // right neighbours
                    neg += __builtin_popcount(cur.d[k] & 0x80808080u);
                    anti += __builtin_popcount((cur.d[k] ^ rn) & 0x80808080u);
                    anti += __builtin_popcount((cur.d[k] ^ dn.d[k]) & 0x80808080u);
                }
            }
            cur = dn;
        }
    }
    // every site contributes 2 bonds; block_accumulate converts counts to (M, E) (sites in units of 32)
    block_accumulate(a.out, anti, neg, units, 32u * a.rows);
}

__global__ void k_zero_n(int64_t* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}

__global__ void k_zero2(int64_t* p) {
    if (threadIdx.x == 0) { p[0] = 0; p[1] = 0; }
}

// One wave per spread set s: dst[s n + k] = the sum of word k (k < n <= 4) over the set's lines; the
// lines are then cleared for the next launches that take the set.
__global__ __launch_bounds__(64) void k_fold_spread(int64_t* sets, int64_t* dst, uint32_t n) {
    const uint32_t lane = threadIdx.x;
    int64_t* const line = sets + (size_t)blockIdx.x * kSpreadSetWords + (size_t)lane * kSpreadLineWords;
    long long v[4];
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) v[k] = k < n ? line[k] : 0;
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k)
        if (k < n) line[k] = 0;
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k)
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    if (lane == 0)
        for (uint32_t k = 0; k < n; ++k) dst[(size_t)blockIdx.x * n + k] = v[k];
}

// ---- hot start: bit (c & 31) of word (c >> 5) & 3 of Philox(c >> 7, r, 0, 0x80000000).
__device__ __forceinline__ uint32_t nibble_to_bytes(uint32_t nib) {
    const uint32_t t = (nib * 0x00204081u) & 0x01010101u;  // bit j -> byte j (no carries)
    return 0x01010101u | (t * 0xFEu);                         // 0x01 for +1, 0xFF for -1
}

// A grid-stride loop over (row, 128-column chunk): a dispatch holds fewer than 2^32 work-items.
__global__ __launch_bounds__(256) void k_init_int8(int8_t* spins, uint32_t L, uint32_t chunks,
                                                   uint64_t n_lanes, uint32_t key0, uint32_t key1) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t lane_id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; lane_id < n_lanes; lane_id += stride) {
    const uint32_t cb = (uint32_t)(lane_id % chunks);
    const uint32_t r = (uint32_t)(lane_id / chunks);
    const Words4 w = philox4x32_10(cb, r, 0u, 0x80000000u, key0, key1);
    const uint32_t words[4] = {w.w0, w.w1, w.w2, w.w3};
    int8_t* p = spins + (size_t)r * L + (size_t)cb * 128u;
    const uint32_t left = L - cb * 128u;                              // columns from this chunk on
    const uint32_t n_words = left >= 128u ? 4u : left / 32u;          // L % 32 == 0
    for (uint32_t i = 0; i < n_words; ++i) {
        uint4* v = reinterpret_cast<uint4*>(p + 32u * i);
        const uint32_t x = words[i];
        v[0] = make_uint4(nibble_to_bytes(x & 15u), nibble_to_bytes((x >> 4) & 15u),
                          nibble_to_bytes((x >> 8) & 15u), nibble_to_bytes((x >> 12) & 15u));
        v[1] = make_uint4(nibble_to_bytes((x >> 16) & 15u), nibble_to_bytes((x >> 20) & 15u),
                          nibble_to_bytes((x >> 24) & 15u), nibble_to_bytes(x >> 28));
    }
    }
}

__global__ __launch_bounds__(256) void k_fill_int8(int8_t* spins, uint64_t n16, uint32_t word) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        reinterpret_cast<uint4*>(spins)[i] = make_uint4(word, word, word, word);
}

// ==========================================================================================
// 1-bit packed layout: plane q holds, for every row r and group g, the word of the 32 colour-q
// sites of row r with j = c >> 1 in [32 g, 32 g + 32), bit p(i) for site i (the bit the site's
// uniform uses), set = spin -1.  Word index (q * L + r) * groups + g.
struct PackedArgs {
    uint32_t* planes;
    uint32_t L, groups, rows, n_lanes;
    uint32_t t, key0, key1;
    Thresholds th;
    int64_t* obs;  // OBS: a spread set (zeroed beforehand) that takes (M, E)
    uint32_t xcd_remap;
    uint32_t falling_prio;  // launch of at most two rounds: lower issue priority along the strip
};

// Half-sweep on the packed layout: a lane owns one group of a strip of `rows` rows and streams
// down it.  Vertical neighbours of row r's colour-Q sites are the other plane's words of rows
// r +- 1 (same group); horizontal ones are the other plane's word of row r and its shift by one
// site, whose edge bit comes from the adjacent group's word.
template <int Q, bool OBS, bool HALF = false>
__global__ __launch_bounds__(256) void k_sweep_packed(PackedArgs a) {
    const uint32_t lane_id = logical_block(blockIdx.x, gridDim.x, a.xcd_remap) * blockDim.x + threadIdx.x;
    const bool active = lane_id < a.n_lanes;
    Counts cnt{0u, 0u};
    if (active) {
        const uint32_t W = a.groups, L = a.L, R = a.rows;
        const uint32_t g = lane_id % W;
        const uint32_t r0 = (lane_id / W) * R;
        const uint32_t gl = g == 0 ? W - 1 : g - 1;
        const uint32_t gr = g + 1 == W ? 0 : g + 1;
        // HALF: the last word of each row holds a half group (sites 0 .. 15)
        const bool half = HALF && gr == 0, left_half = HALF && gl + 1 == W;
        const uint32_t valid = half ? kHalfSites : 0xFFFFFFFFu;
        uint32_t* const pq = a.planes + (size_t)Q * L * W;        // sites being updated
        const uint32_t* const po = a.planes + (size_t)(1 - Q) * L * W;  // other colour
        auto wrapr = [&](uint32_t r) { return r >= L ? r - L : r; };
        uint32_t bprev = po[(size_t)(r0 == 0 ? L - 1 : r0 - 1) * W + g];
        uint32_t bcur = po[(size_t)r0 * W + g];
        uint32_t acur = pq[(size_t)r0 * W + g];
#pragma unroll 1
        for (uint32_t s = 0; s < R; s += 2) {
            const uint32_t r = r0 + s, r1 = r + 1, r2 = wrapr(r + 2);
            // row r: colour-Q sites at column parity Q (r even); row r + 1: parity 1 - Q
            const uint32_t bn = po[(size_t)r1 * W + g];
            const uint32_t a1 = pq[(size_t)r1 * W + g];
            const uint32_t bn2 = po[(size_t)r2 * W + g];
            const uint32_t a2 = s + 2 < R ? pq[(size_t)r2 * W + g] : 0u;
            const uint32_t e0 = Q == 1 ? po[(size_t)r * W + gr] : po[(size_t)r * W + gl];
            const uint32_t e1 = Q == 1 ? po[(size_t)r1 * W + gl] : po[(size_t)r1 * W + gr];
            // parity 1 (Q = 1 on even rows): right neighbour is site j + 1 -> shift_next with the
            // next group's site 0 (bit 0); parity 0: left neighbour j - 1 -> shift_prev with the
            // previous group's site 31 (bit 31)
            const uint32_t hs0 = Q == 1 ? (half ? shift_next_half(bcur, e0 & 1u) : shift_next(bcur, e0 & 1u))
                                        : shift_prev(bcur, last_site_bit(e0, left_half));
            uint32_t F = decide<Q, OBS>(acur, bprev, bn, bcur, hs0, bcur, a.th, g, r, a.t, a.key0, a.key1, cnt, valid);
            pq[(size_t)r * W + g] = acur ^ F;
            const uint32_t hs1 = Q == 1 ? shift_prev(bn, last_site_bit(e1, left_half))
                                        : (half ? shift_next_half(bn, e1 & 1u) : shift_next(bn, e1 & 1u));
            F = decide<Q, OBS>(a1, bcur, bn2, bn, hs1, bn, a.th, g, r1, a.t, a.key0, a.key1, cnt, valid);
            pq[(size_t)r1 * W + g] = a1 ^ F;
            bprev = bn;
            bcur = bn2;
            acur = a2;
        }
    }
    // sites in units of 32: a lane covers two per row, one in a half group
    const uint32_t units = !active ? 0u : (HALF && lane_id % a.groups + 1 == a.groups) ? 1u : 2u;
    if (OBS) block_accumulate(spread_line(a.obs, blockIdx.x), cnt.anti, cnt.neg, units, 32u * a.rows);
}

// Half-sweep on the packed layout with the ties of four rows settled together.  All colour-Q sites
// of a half-sweep are independent, so a lane takes rows r .. r + 3 of its strip at a time, draws
// the first two Philox blocks of each row's word, queues the words still holding tied sites and
// settles them with the other lanes' (as in the two-sweep pass).  Same uniforms and results as
// k_sweep_packed.  rows % 4 == 0; lanes past n_lanes shadow the last lane without storing.
// UROW (groups % 64 == 0): every wave lies in one strip, so its rows are uniform and the Philox rounds
// that depend only on (row, sweep, colour) run on the scalar unit.
template <int Q, bool OBS, bool HALF = false, bool O32 = false, bool UROW = false>
__global__ __launch_bounds__(512) void k_sweep_packed_q(PackedArgs a) {
    extern __shared__ uint4 packed_lds[];
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    uint4* const mine = packed_lds + (tid >> 6) * (kTieQueueBytes / 16u);
    const TieQueue q{reinterpret_cast<uint32_t*>(mine), mine + 256};
    const uint32_t raw_id = logical_block(blockIdx.x, gridDim.x, a.xcd_remap) * blockDim.x + tid;
    const bool active = raw_id < a.n_lanes;
    const uint32_t lane_id = active ? raw_id : a.n_lanes - 1u;
    Counts cnt{0u, 0u};
    const uint32_t W = a.groups, L = a.L, R = a.rows;
    const uint32_t g = lane_id % W;
    const uint32_t r0 = UROW ? __builtin_amdgcn_readfirstlane((lane_id / W) * R) : (lane_id / W) * R;
    const uint32_t gl = g == 0 ? W - 1 : g - 1;
    const uint32_t gr = g + 1 == W ? 0 : g + 1;
    // HALF: the last word of each row holds a half group (sites 0 .. 15)
    const bool half = HALF && gr == 0, left_half = HALF && gl + 1 == W;
    const uint32_t valid = half ? kHalfSites : 0xFFFFFFFFu;
    uint32_t* const pq = a.planes + (size_t)Q * L * W;              // sites being updated
    const uint32_t* const po = a.planes + (size_t)(1 - Q) * L * W;  // other colour
    // O32 (a plane of at most 4 GiB): word (r, gg) of a plane at a 32-bit byte offset from its base,
    // so that a load takes the base from scalar registers and one 32-bit offset per lane
    auto word_at = [&](const uint32_t* plane, uint32_t r, uint32_t gg) -> const uint32_t* {
        if (O32) return reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(plane) + (r * W + gg) * 4u);
        return plane + (size_t)r * W + gg;
    };
    // the same from a row's word offset r W (O32)
    auto word_off = [&](const uint32_t* plane, uint32_t rw, uint32_t gg) -> const uint32_t* {
        return reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(plane) + (rw + gg) * 4u);
    };
    // row r + i (r even): colour-Q sites at column parity Q for even i, 1 - Q for odd i; parity 1
    // takes the right group's site 0 as the far horizontal neighbour, parity 0 the left group's
    // site 31
    uint32_t bprev = *word_at(po, r0 == 0 ? L - 1 : r0 - 1, g);
    uint32_t bcur = *word_at(po, r0, g);
#pragma unroll 1
    for (uint32_t s = 0; s < R; s += 4) {
        // In a launch of few rounds, waves that are further down their strips yield issue slots to
        // those behind, so that fewer waves are left running alone at the end.
        if (a.falling_prio) {
            switch ((4u * s) / R) {
                case 0: __builtin_amdgcn_s_setprio(3); break;
                case 1: __builtin_amdgcn_s_setprio(2); break;
                case 2: __builtin_amdgcn_s_setprio(1); break;
                default: __builtin_amdgcn_s_setprio(0); break;
            }
        }
        const uint32_t r = r0 + s;
        uint32_t b[6], w[4], e[4];
        b[0] = bprev;
        b[1] = bcur;
        if (O32) {
            // row offsets by additions from r W; only row r + 4 == L wraps (to row 0)
            const uint32_t rw = r * W;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t ri_w = rw + (uint32_t)i * W;
                const uint32_t rn_w = r + (uint32_t)i + 1u == L ? 0u : ri_w + W;
                b[i + 2] = *word_off(po, rn_w, g);
                w[i] = *word_off(pq, ri_w, g);
                const bool right = (Q == 1) == ((i & 1) == 0);
                e[i] = *word_off(po, ri_w, right ? gr : gl);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t ri = r + (uint32_t)i, rn = ri + 1u >= L ? ri + 1u - L : ri + 1u;
                b[i + 2] = *word_at(po, rn, g);
                w[i] = *word_at(pq, ri, g);
                const bool right = (Q == 1) == ((i & 1) == 0);
                e[i] = *word_at(po, ri, right ? gr : gl);
            }
        }
        q.res[lane] = make_uint4(0u, 0u, 0u, 0u);
        uint32_t n = 0u;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const bool right = (Q == 1) == ((i & 1) == 0);
            const uint32_t side = b[i + 1];
            const uint32_t hs = right ? (half ? shift_next_half(side, e[i] & 1u) : shift_next(side, e[i] & 1u))
                                      : shift_prev(side, last_site_bit(e[i], left_half));
            const uint32_t x1 = w[i] ^ b[i], x2 = w[i] ^ b[i + 2], x3 = w[i] ^ side, x4 = w[i] ^ hs;
            const uint32_t o12 = x1 | x2, o34 = x3 | x4;
            // three-input logic as explicit v_bitop3 (issued at twice the rate of the v_or3_b32 /
            // v_and_or_b32 the compiler forms; the kernel is bound by issue), one uniform mask each:
            // ge2 = (x1 & x2) | (x3 & x4) | (o12 & o34), flip = ge2 | (any & f2) | (~any & f4)
            const uint32_t ge2 = and_or3(o12, o34, and_or3(x3, x4, x1 & x2)) & valid;
            const uint32_t any = o12 | o34;
            const uint32_t flip = __builtin_amdgcn_bitop3_b32(any, a.th.f4, and_or3(any, a.th.f2, ge2), 0xAE) & valid;
            const uint32_t sel2 = __builtin_amdgcn_bitop3_b32(any, flip, 0u, 0x30) & valid;  // a & ~b
            uint32_t acc = flip, tied = ~flip & valid;
#pragma unroll
            for (uint32_t m = 0; m < 2; ++m) {
                if (!wave_any(tied != 0u)) break;
                compare_planes<true>(acc, tied, sel2,
                               philox4x32_10<2, UROW ? 3 : 1>(g, r + (uint32_t)i, a.t, 2u * m + (uint32_t)Q, a.key0, a.key1),
                               a.th, m);
            }
            w[i] ^= acc;
            tq_push(q, n, tied, sel2, r + (uint32_t)i, (uint32_t)i | (lane << 2) | (g << 8));
        }
        tq_settle<Q>(q, n, a.th, a.t, a.key0, a.key1, lane);
        const uint4 res = q.res[lane];
        w[0] ^= res.x;
        w[1] ^= res.y;
        w[2] ^= res.z;
        w[3] ^= res.w;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (active) *const_cast<uint32_t*>(word_at(pq, r + (uint32_t)i, g)) = w[i];
            if (OBS) {
                const bool right = (Q == 1) == ((i & 1) == 0);
                const uint32_t side = b[i + 1];
                const uint32_t hs = right ? (half ? shift_next_half(side, e[i] & 1u) : shift_next(side, e[i] & 1u))
                                          : shift_prev(side, last_site_bit(e[i], left_half));
                cnt.anti += __builtin_popcount((w[i] ^ b[i]) & valid) + __builtin_popcount((w[i] ^ b[i + 2]) & valid) +
                            __builtin_popcount((w[i] ^ side) & valid) + __builtin_popcount((w[i] ^ hs) & valid);
                cnt.neg += __builtin_popcount(w[i] & valid) + __builtin_popcount(side & valid);
            }
        }
        bprev = b[4];
        bcur = b[5];
    }
    // sites in units of 32: a lane covers two per row, one in a half group
    const uint32_t units = !active ? 0u : half ? 1u : 2u;
    if (OBS) block_accumulate(spread_line(a.obs, blockIdx.x), active ? cnt.anti : 0u, active ? cnt.neg : 0u, units,
                              32u * a.rows);
}

// (M, E) of a packed lattice: every bond has exactly one black (q = 0) end, so the black sites'
// anti-aligned neighbour counts cover all 2 L^2 bonds once.  A grid-stride loop over (row, group)
// words: a bounded grid keeps the final atomics few at any L.
__global__ __launch_bounds__(256) void k_observables_packed(const uint32_t* planes, uint32_t L, uint32_t groups,
                                                            uint64_t n_lanes, int64_t* out) {
    uint32_t anti = 0, neg = 0, words = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t lane_id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; lane_id < n_lanes; lane_id += stride) {
        const uint32_t W = groups;
        const uint32_t g = (uint32_t)(lane_id % W), r = (uint32_t)(lane_id / W);
        const uint32_t gl = g == 0 ? W - 1 : g - 1, gr = g + 1 == W ? 0 : g + 1;
        // a half group (16 sites) ends each row when L is an odd multiple of 32
        const bool odd32 = (L & 63u) != 0, half = odd32 && gr == 0, left_half = odd32 && gl + 1 == W;
        const uint32_t valid = half ? kHalfSites : 0xFFFFFFFFu;
        const uint32_t* p0 = planes;
        const uint32_t* p1 = planes + (size_t)L * W;
        const uint32_t up = r == 0 ? L - 1 : r - 1, dn = r + 1 == L ? 0 : r + 1;
        const uint32_t b = p0[(size_t)r * W + g];
        const uint32_t w = p1[(size_t)r * W + g];
        // black sites of row r sit at column parity r & 1
        const uint32_t right0 = p1[(size_t)r * W + gr] & 1u;
        const uint32_t hs = (r & 1u) ? (half ? shift_next_half(w, right0) : shift_next(w, right0))
                                     : shift_prev(w, last_site_bit(p1[(size_t)r * W + gl], left_half));
        anti += __builtin_popcount((b ^ p1[(size_t)up * W + g]) & valid) +
                __builtin_popcount((b ^ p1[(size_t)dn * W + g]) & valid) + __builtin_popcount((b ^ w) & valid) +
                __builtin_popcount((b ^ hs) & valid);
        neg += __builtin_popcount(b & valid) + __builtin_popcount(w & valid);
        words += half ? 1u : 2u;
    }
    // `words` counts 32-site units (two per word, one per half word).  With the grid capped at 16384
    // blocks of 256 threads a thread takes at most 2^12 words (L = 2^20), so its counts stay below 2^19
    // and a wave's below 2^25 (32-bit sums)
    block_accumulate(out, anti, neg, words, 32u);
}

// int8 -> packed: lane per (row, group)
__global__ __launch_bounds__(256) void k_pack(const int8_t* spins, uint32_t* planes, uint32_t L, uint32_t groups,
                                              uint64_t n_lanes) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t lane_id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; lane_id < n_lanes; lane_id += stride) {
    const uint32_t g = (uint32_t)(lane_id % groups), r = (uint32_t)(lane_id / groups);
    // the last group of a row whose length is an odd multiple of 32 is a half group (sites 0 .. 15);
    // its other bits are kept zero
    const bool half = (L & 63u) != 0 && g + 1 == groups;
    Row row;
    if (half) load_row_half(row, spins + (size_t)r * L + (size_t)g * 64u);
    else load_row(row, spins + (size_t)r * L + (size_t)g * 64u);
    const uint32_t valid = half ? kHalfSites : 0xFFFFFFFFu;
    const uint32_t even = site_bits<0>(row) & valid, odd = site_bits<1>(row) & valid;
    // colour q of row r sits at column parity (r + q) & 1
    planes[(size_t)r * groups + g] = (r & 1u) ? odd : even;                          // q = 0
    planes[((size_t)L + r) * groups + g] = (r & 1u) ? even : odd;                    // q = 1
    }
}

// cold start in the packed layout: every word `word`, masked to its sites in a half group
__global__ __launch_bounds__(256) void k_fill_packed(uint32_t* planes, uint64_t n, uint32_t groups, uint32_t half,
                                                     uint32_t word) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        planes[i] = half && i % groups + 1 == groups ? word & kHalfSites : word;
}

// packed -> int8
__global__ __launch_bounds__(256) void k_unpack(const uint32_t* planes, int8_t* spins, uint32_t L, uint32_t groups,
                                                uint64_t n_lanes) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t lane_id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; lane_id < n_lanes; lane_id += stride) {
    const uint32_t g = (uint32_t)(lane_id % groups), r = (uint32_t)(lane_id / groups);
    const uint32_t q0 = planes[(size_t)r * groups + g], q1 = planes[((size_t)L + r) * groups + g];
    const uint32_t even = (r & 1u) ? q1 : q0, odd = (r & 1u) ? q0 : q1;
    Row row;
    // dword 2k + h: bytes 0, 2 are even-column sites at bits k + 8h, k + 8h + 16; bytes 1, 3 the
    // odd-column ones at the same bits of the other word.  Sign-extending permute selectors 8..11
    // replicate bits 15 / 31 of each source into whole bytes.
#pragma unroll
    for (int k = 0; k < 8; ++k) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t sh = 15 - k - 8 * h;
            row.d[2 * k + h] = perm(odd << sh, even << sh, 0x0B090A08u) | 0x01010101u;
        }
    }
    if ((L & 63u) != 0 && g + 1 == groups) store_row_half(spins + (size_t)r * L + (size_t)g * 64u, row);
    else store_row(spins + (size_t)r * L + (size_t)g * 64u, row, false);
    }
}

// packed hot start: the int8 hot start's bits for one group, regrouped by colour
__global__ __launch_bounds__(256) void k_init_packed(uint32_t* planes, uint32_t L, uint32_t groups, uint64_t n_lanes,
                                                     uint32_t key0, uint32_t key1) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t lane_id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; lane_id < n_lanes; lane_id += stride) {
    const uint32_t g = (uint32_t)(lane_id % groups), r = (uint32_t)(lane_id / groups);
    const Words4 w = philox4x32_10(g >> 1, r, 0u, 0x80000000u, key0, key1);
    const uint32_t lo = (g & 1u) ? w.w2 : w.w0, hi = (g & 1u) ? w.w3 : w.w1;  // columns 0-31, 32-63
    Row row;
#pragma unroll
    for (int d = 0; d < 16; ++d) {
        const uint32_t src = d < 8 ? lo : hi;
        row.d[d] = nibble_to_bytes((src >> (4 * (d & 7))) & 15u);
    }
    const uint32_t valid = (L & 63u) != 0 && g + 1 == groups ? kHalfSites : 0xFFFFFFFFu;  // half group
    const uint32_t even = site_bits<0>(row) & valid, odd = site_bits<1>(row) & valid;
    planes[(size_t)r * groups + g] = (r & 1u) ? odd : even;
    planes[((size_t)L + r) * groups + g] = (r & 1u) ? even : odd;
    }
}

// ==========================================================================================
// Batched replicas: one workgroup per replica (L = 32 or L % 64 == 0, L <= 512), the lattice in LDS as
// the two colour planes of the packed layout, all sweeps of the run in one launch.  Every replica
// uses the single-lattice chain's random numbers (its own seed, the same counters), so each one is
// bit-identical to ising_sweep_packed on that replica alone.
struct BatchReplica {
    uint32_t L;          // linear size
    uint32_t W;          // words per row per colour: L / 64, or 1 for L = 32 (16 sites per word)
    uint32_t key0, key1;
    uint32_t t0;         // sweep index of the first sweep of this run
    uint32_t ordered;    // 1 when beta > beta_c (start mode 3 begins from the ordered state)
    Thresholds th;
    uint32_t pad2;
    uint64_t state_off;  // word offset of this replica's planes in the state buffer
};


// Rows of 16 same-colour sites (L = 32): the word wraps onto itself after site 15, and only
// sites 0..15 (bits 0-3 of each byte in site order) exist.
__device__ __forceinline__ uint32_t shift_next16(uint32_t y) {
    const uint32_t top = ((y >> 1) & 0x07u) | ((y & 1u) << 3);
    return perm(top, y, 0x04010302u);
}
__device__ __forceinline__ uint32_t shift_prev16(uint32_t y) {
    const uint32_t low = ((y >> 23) & 0x0Eu) | ((y >> 27) & 1u);
    return perm(y, low, 0x05040600u);
}

// Hot-start words of row r, group g of an L x L lattice: (colour-0 word, colour-1 word).
__device__ __forceinline__ void hot_start_words(uint32_t L, uint32_t r, uint32_t g, uint32_t key0, uint32_t key1,
                                                uint32_t& w0, uint32_t& w1) {
    const Words4 w = philox4x32_10(g >> 1, r, 0u, 0x80000000u, key0, key1);
    const uint32_t lo = (g & 1u) ? w.w2 : w.w0, hi = (g & 1u) ? w.w3 : w.w1;  // columns 0-31, 32-63
    Row row;
#pragma unroll
    for (int d = 0; d < 16; ++d) {
        const uint32_t src = d < 8 ? lo : (L >= 64 ? hi : 0u);
        row.d[d] = nibble_to_bytes((src >> (4 * (d & 7))) & 15u);
    }
    const uint32_t even = site_bits<0>(row), odd = site_bits<1>(row);
    w0 = (r & 1u) ? odd : even;
    w1 = (r & 1u) ? even : odd;
}

// One entry of a workgroup's work list: a whole replica (depth 0, its rows wrap inside LDS) or
// one slab of a split replica, rows [row0, row0 + rows).  A slab also holds `depth` rows beyond
// either edge (halo rows, local rows 0 .. depth - 1 and depth + rows ..) and updates rows 1 ..
// rows + 2 depth - 2 at every colour update: each update leaves one more outer row stale on
// either side, so its own rows stay exact for `depth` updates, after which neighbouring slabs
// trade their outer `depth` rows through the exchange area.
struct BatchUnit {
    uint32_t rep;        // replica index
    uint32_t slab, slabs;
    uint32_t row0, rows;
    uint32_t depth;      // halo rows per side (= colour updates between exchanges); 0 unsplit
    uint32_t lag;        // measurement sweeps between a sweep and the combination of its counts
    uint32_t lds;        // word offset of its two colour planes in the workgroup's LDS
    uint32_t first;      // first wave slot (64 words) of its words in one colour update of the workgroup
    uint32_t xfirst;     // first flat index of its words in one exchange of the workgroup
    uint64_t xoff;       // offset (64-bit words) of the replica's exchange area
};

// A workgroup's work list: units [begin, end) of the unit table.
struct BatchGroup {
    uint32_t begin, end;
    uint32_t words;      // wave slots (64 words each) of one colour update over all its units
    uint32_t xwords;     // words of one exchange over all its units
};

constexpr uint32_t kMaxSlabs = 8;
constexpr uint32_t kMaxDepth = 4;
constexpr uint32_t kMaxUnits = 32;           // units per workgroup
constexpr uint32_t kCountSlots = 32;         // ring of per-slab count slots (> 2 x the largest lag)
constexpr uint32_t kPollLimit = 1u << 20;    // polls of one tagged word before the run gives up

__host__ __device__ constexpr uint32_t unit_words(uint32_t rows, uint32_t depth, uint32_t W) {
    return (depth ? rows + 2u * depth - 2u : rows) * W;
}
__host__ __device__ constexpr uint32_t unit_xwords(uint32_t depth, uint32_t W) { return 2u * depth * 2u * W; }
__host__ __device__ constexpr uint32_t unit_plane(uint32_t rows, uint32_t depth, uint32_t W) {
    return (rows + 2u * depth) * W;
}

// 64-bit words of one replica's exchange area: two alternating slots of every slab's outer rows
// (2 sides x depth rows x 2 colours), then kCountSlots x slabs x (anti, neg) counts.  Every word
// is (tag << 32) | value, written and read as one atomic, so a reader that sees the tag it waits
// for sees its value.
__host__ __device__ constexpr uint64_t exchange_words(uint32_t W) {
    return 2ull * kMaxSlabs * 2u * kMaxDepth * 2u * W + (uint64_t)kCountSlots * kMaxSlabs * 2u;
}

__device__ __forceinline__ uint64_t* edge_word(uint64_t* x, uint32_t W, uint32_t slot, uint32_t slab, uint32_t side,
                                               uint32_t k, uint32_t c, uint32_t g) {
    return x + ((((uint64_t)slot * kMaxSlabs + slab) * 2u + side) * kMaxDepth * 2u + k * 2u + c) * W + g;
}

__device__ __forceinline__ uint64_t* count_word(uint64_t* x, uint32_t W, uint32_t j, uint32_t slab) {
    return x + 2ull * kMaxSlabs * 2u * kMaxDepth * 2u * W + ((uint64_t)(j % kCountSlots) * kMaxSlabs + slab) * 2u;
}

__device__ __forceinline__ void put_tagged(uint64_t* p, uint32_t tag, uint32_t v) {
    __hip_atomic_store(p, ((uint64_t)tag << 32) | v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait (bounded) until *p carries `tag`; false when the wait gave up.
__device__ __forceinline__ bool get_tagged(const uint64_t* p, uint32_t tag, uint32_t& v) {
    for (uint32_t k = 0; k < kPollLimit; ++k) {
        const uint64_t x = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((uint32_t)(x >> 32) == tag) { v = (uint32_t)x; return true; }
        __builtin_amdgcn_s_sleep(1);
    }
    return false;
}

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Colour update of every unit of the workgroup (colour Q, sweep i).  Each unit's words are
// padded to whole waves ("slots" of 64 words): wave w takes slots w, w + waves, ..., so a wave
// always works inside one unit, whose parameters it holds in scalar registers.  Counts of owned
// rows go to cnt[unit] with OBS, one wave sum per unit.
template <int Q, bool OBS>
__device__ __forceinline__ void batch_update(uint32_t* lds, const BatchUnit* us, const BatchReplica* rs, uint32_t nu,
                                             uint32_t slots, uint32_t i, uint32_t (*cnt)[2]) {
    const uint32_t waves = blockDim.x >> 6, lane = threadIdx.x & 63u;
    uint32_t u = 0;
    uint32_t uend = nu > 1 ? us[1].first : slots;
    Counts c{0u, 0u};
    auto flush = [&]() {
        if (OBS) {
            const uint32_t A = wave_sum(c.anti), Nn = wave_sum(c.neg);
            if (lane == 0 && (A | Nn)) { atomicAdd(&cnt[u][0], A); atomicAdd(&cnt[u][1], Nn); }
            c = Counts{0u, 0u};
        }
    };
    for (uint32_t sl = threadIdx.x >> 6; sl < slots; sl += waves) {
        while (sl >= uend) {
            flush();
            ++u;
            uend = u + 1 < nu ? us[u + 1].first : slots;
        }
        const BatchUnit& x = us[u];
        const BatchReplica& rp = rs[u];
        const uint32_t W = uni(rp.W), L = uni(rp.L), K = uni(x.depth), rows = uni(x.rows);
        const uint32_t n = (K ? rows + 2u * K - 2u : rows) * W;
        const uint32_t local = (sl - uni(x.first)) * 64u + lane;
        if (local < n) {
            const uint32_t pw = (rows + 2u * K) * W, base = uni(x.lds);
            uint32_t* pq = lds + base + Q * pw;
            const uint32_t* po = lds + base + (1 - Q) * pw;
            const Thresholds th{uni(rp.th.t2), uni(rp.th.t4), uni(rp.th.f2), uni(rp.th.f4), uni(rp.th.blocks)};
            const uint32_t t = uni(rp.t0) + i, key0 = uni(rp.key0), key1 = uni(rp.key1);
            uint32_t lr, lup, ldn, r;
            bool own;
            if (K == 0) {
                lr = local / W;
                lup = lr == 0 ? rows - 1 : lr - 1;
                ldn = lr + 1 == rows ? 0 : lr + 1;
                r = lr;
                own = true;
            } else {
                lr = local / W + 1u;
                lup = lr - 1;
                ldn = lr + 1;
                r = (uni(x.row0) + L - K + lr) % L;
                own = lr >= K && lr < K + rows;
            }
            const uint32_t g = local - (K ? lr - 1u : lr) * W;
            const uint32_t valid = L >= 64 ? 0xFFFFFFFFu : 0x0F0F0F0Fu;
            const uint32_t w = lr * W + g;
            const uint32_t a = pq[w], side = po[w];
            const uint32_t up = po[lup * W + g], down = po[ldn * W + g];
            const uint32_t o = (r + Q) & 1u;   // column parity of this row's colour-Q sites
            uint32_t hs;
            if (L >= 64) {
                const uint32_t gl = g == 0 ? W - 1 : g - 1, gr = g + 1 == W ? 0 : g + 1;
                hs = o ? shift_next(side, po[lr * W + gr] & 1u) : shift_prev(side, po[lr * W + gl] >> 31);
            } else {
                hs = o ? shift_next16(side) : shift_prev16(side);
            }
            Counts cw{0u, 0u};
            const uint32_t F = decide<Q, OBS>(a, up, down, side, hs, side, th, g, r, t, key0, key1, cw, valid);
            if (OBS && own) { c.anti += cw.anti; c.neg += cw.neg; }
            pq[w] = a ^ F;
        }
    }
    flush();
}

// Exchange e of the split units (after colour updates e depth .. (e + 1) depth - 1): publish
// each slab's outer `depth` rows of both colours (slot e mod 2, tag e + 1), then take the
// neighbouring slabs' as its halo rows.  A slab overwrites a slot only after taking its
// neighbours' next publication, which they make after reading this one, so two alternating slots
// suffice.  Returns false if a wait gave up.
__device__ __forceinline__ bool batch_exchange(uint32_t* lds, const BatchUnit* us, const BatchReplica* rs, uint32_t nu,
                                               uint32_t xwords, uint64_t* exchange, uint32_t e) {
    const uint32_t slot = e & 1u, tag = e + 1u;
    bool ok = true;
    for (int pass = 0; pass < 2; ++pass) {
        uint32_t u = 0;
        uint32_t uend = nu > 1 ? us[1].xfirst : xwords;
        for (uint32_t f = threadIdx.x; f < xwords; f += blockDim.x) {
            while (f >= uend) {
                ++u;
                uend = u + 1 < nu ? us[u + 1].xfirst : xwords;
            }
            const BatchUnit& x = us[u];
            const uint32_t W = rs[u].W, K = x.depth, rows = x.rows, pw = unit_plane(rows, K, W);
            const uint32_t i = f - x.xfirst;
            const uint32_t g = i % W, c = (i / W) & 1u, k = (i / (2u * W)) % K, side = i / (2u * W * K);
            uint64_t* xchg = exchange + x.xoff;
            uint32_t* plane = lds + x.lds + c * pw;
            if (pass == 0) {
                // side 0: own rows 0 .. K - 1 (local K + k); side 1: own rows rows - K .. rows - 1
                put_tagged(edge_word(xchg, W, slot, x.slab, side, k, c, g), tag, plane[(side == 0 ? K + k : rows + k) * W + g]);
            } else {
                // side 0: halo above = the previous slab's last rows; side 1: halo below = the next
                // slab's first rows
                const uint32_t prev = x.slab == 0 ? x.slabs - 1 : x.slab - 1;
                const uint32_t next = x.slab + 1 == x.slabs ? 0 : x.slab + 1;
                const uint64_t* src = side == 0 ? edge_word(xchg, W, slot, prev, 1, k, c, g)
                                                : edge_word(xchg, W, slot, next, 0, k, c, g);
                uint32_t v = 0;
                ok = get_tagged(src, tag, v) && ok;
                plane[(side == 0 ? k : K + rows + k) * W + g] = v;
            }
        }
    }
    return ok;
}

// FP64 moment sums of one sample, each operation rounded as written (no fused multiply-add), so
// the sums equal a plain sequential evaluation in the same order.
__device__ __forceinline__ void accumulate_moments(int64_t M, int64_t E, double n_sites, double& s_abs, double& s_m2,
                                                   double& s_m4, double& s_e, double& s_e2) {
#pragma clang fp contract(off)
    const double m = (double)M / n_sites, e = (double)E / n_sites, m2 = m * m;
    s_abs += fabs(m);
    s_m2 += m2;
    s_m4 += m2 * m2;
    s_e += e;
    s_e2 += e * e;
}

__device__ __forceinline__ void store_moments(double* mo, uint32_t n, double s_abs, double s_m2, double s_m4,
                                              double s_e, double s_e2) {
#pragma clang fp contract(off)
    const double k = (double)n;
    mo[0] = s_abs / k;
    mo[1] = s_m2 / k;
    mo[2] = s_m4 / k;
    mo[3] = s_e / k;
    mo[4] = s_e2 / k;
}

// start: 0 = hot start from the seed, 1 = cold start (all +1), 2 = continue from `state`,
// 3 = cold start for replicas with beta above the critical value, hot start otherwise.
// One workgroup per work list; `lds` (dynamic) holds both colour planes of every unit of the list.
// `depth`: colour updates between exchanges when the list has split units (0 when none does).  A
// split replica's (M, E) of a measurement sweep is the sum of its slabs' counts, combined by its
// slab 0 `lag` sweeps later (or at the end); a run in which a wait gave up leaves NaN moments.
// Per-call values of a batch run.  k_batch reads them from the workspace, so that one captured graph
// serves every call with the same plan; k_batch_set_run writes them on the caller's stream first.
struct BatchRun {
    uint32_t start, n_therm, n_meas, pad;
    int64_t* trace;    // (M, E) of every measurement sweep, replica-major, or NULL
    double* moments;   // FP64 moments per replica, or NULL
};

__global__ void k_batch_set_run(BatchRun* run, BatchRun v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *run = v;
}

__global__ __launch_bounds__(1024) void k_batch(const BatchReplica* table, const BatchGroup* groups,
                                                const BatchUnit* units, uint32_t* state, uint64_t* exchange,
                                                uint32_t depth, const BatchRun* run) {
    extern __shared__ uint32_t lds[];
    const uint32_t start = run->start, n_therm = run->n_therm, n_meas = run->n_meas;
    int64_t* const trace = run->trace;
    double* const moments = run->moments;
    __shared__ BatchUnit us[kMaxUnits];
    __shared__ BatchReplica rs[kMaxUnits];
    __shared__ uint32_t cnt[kMaxUnits][2];
    __shared__ double acc[kMaxUnits][5];
    __shared__ uint32_t took[kMaxUnits];
    const BatchGroup grp = groups[blockIdx.x];
    const uint32_t nu = grp.end - grp.begin;
    for (uint32_t u = threadIdx.x; u < nu; u += blockDim.x) {
        us[u] = units[grp.begin + u];
        rs[u] = table[us[u].rep];
        cnt[u][0] = cnt[u][1] = 0u;
        for (int k = 0; k < 5; ++k) acc[u][k] = 0.0;
        took[u] = 0u;
    }
    __syncthreads();
    // every unit's rows and halo rows (global rows row0 - depth .. row0 + rows + depth - 1)
    for (uint32_t u = 0; u < nu; ++u) {
        const BatchUnit& x = us[u];
        const BatchReplica& rp = rs[u];
        const uint32_t W = rp.W, L = rp.L, words = L * W, pw = unit_plane(x.rows, x.depth, W);
        const uint32_t mode = start == 3 ? (rp.ordered ? 1u : 0u) : start;
        const uint32_t* gstate = state + rp.state_off;
        for (uint32_t w = threadIdx.x; w < pw; w += blockDim.x) {
            const uint32_t lr = w / W, g = w - lr * W;
            const uint32_t r = (x.row0 + L - x.depth + lr) % L;
            uint32_t w0 = 0u, w1 = 0u;
            if (mode == 0) hot_start_words(L, r, g, rp.key0, rp.key1, w0, w1);
            else if (mode == 2) { w0 = gstate[r * W + g]; w1 = gstate[words + r * W + g]; }
            lds[x.lds + w] = w0;
            lds[x.lds + pw + w] = w1;
        }
    }
    __syncthreads();
    bool ok = true;        // this thread's waits so far
    bool aborted = false;  // some wait of the workgroup gave up
    // (M, E) of measurement sweep j of unit u's replica (slab 0, or the whole replica)
    auto take = [&](uint32_t u, int64_t M, int64_t E, uint32_t j) {
        const BatchReplica& rp = rs[u];
        if (trace) {
            int64_t* tr = trace + 2 * ((size_t)us[u].rep * n_meas + j);
            tr[0] = M;
            tr[1] = E;
        }
        accumulate_moments(M, E, (double)rp.L * (double)rp.L, acc[u][0], acc[u][1], acc[u][2], acc[u][3],
                           acc[u][4]);
    };
    auto combine = [&](uint32_t u, uint32_t j) {
        const BatchUnit& x = us[u];
        const int64_t sites = (int64_t)rs[u].L * rs[u].L;
        uint64_t A = 0, Nn = 0;
        uint64_t* xchg = exchange + x.xoff;
        for (uint32_t p = 0; p < x.slabs && ok; ++p) {
            uint32_t a = 0, n = 0;
            const uint64_t* cw = count_word(xchg, rs[u].W, j, p);
            ok = get_tagged(cw, j + 1u, a) && get_tagged(cw + 1, j + 1u, n);
            A += a;
            Nn += n;
        }
        take(u, sites - 2 * (int64_t)Nn, 2 * (int64_t)A - 2 * sites, j);
    };
    const uint32_t H = 2u * (n_therm + n_meas);
    for (uint32_t h = 0; h < H; ++h) {
        const uint32_t i = h >> 1;
        const bool obs = (h & 1u) && i >= n_therm;
        if (!(h & 1u)) batch_update<1, false>(lds, us, rs, nu, grp.words, i, cnt);
        else if (!obs) batch_update<0, false>(lds, us, rs, nu, grp.words, i, cnt);
        else batch_update<0, true>(lds, us, rs, nu, grp.words, i, cnt);
        __syncthreads();
        const bool exch = depth > 0 && (h + 1u) % depth == 0 && h + 1u < H;
        if (exch) ok = batch_exchange(lds, us, rs, nu, grp.xwords, exchange, h / depth) && ok;
        if (obs) {
            const uint32_t j = i - n_therm;
            for (uint32_t u = threadIdx.x; u < nu; u += blockDim.x) {
                const BatchUnit& x = us[u];
                const uint32_t A = cnt[u][0], Nn = cnt[u][1];
                cnt[u][0] = cnt[u][1] = 0u;   // next added to after the next colour update's barrier
                if (x.slabs == 1) {
                    const int64_t sites = (int64_t)rs[u].L * rs[u].L;
                    take(u, sites - 2 * (int64_t)Nn, 2 * (int64_t)A - 2 * sites, j);
                } else {
                    uint64_t* cw = count_word(exchange + x.xoff, rs[u].W, j, x.slab);
                    put_tagged(cw, j + 1u, A);
                    put_tagged(cw + 1, j + 1u, Nn);
                    if (x.slab == 0 && j >= x.lag) combine(u, took[u]++);
                }
            }
        }
        // halo rows and the abort decision settled for every thread
        if (depth > 0 && (exch || obs) && __syncthreads_or(!ok)) { aborted = true; break; }
    }
    if (!aborted)
        for (uint32_t u = threadIdx.x; u < nu; u += blockDim.x)
            if (us[u].slabs > 1 && us[u].slab == 0)
                while (ok && took[u] < n_meas) combine(u, took[u]++);
    // every unit's own rows (local rows depth .. depth + rows - 1) back to the state buffer
    for (uint32_t u = 0; u < nu; ++u) {
        const BatchUnit& x = us[u];
        const BatchReplica& rp = rs[u];
        const uint32_t W = rp.W, words = rp.L * W, pw = unit_plane(x.rows, x.depth, W);
        uint32_t* gstate = state + rp.state_off;
        for (uint32_t w = threadIdx.x; w < x.rows * W; w += blockDim.x) {
            gstate[x.row0 * W + w] = lds[x.lds + x.depth * W + w];
            gstate[words + x.row0 * W + w] = lds[x.lds + pw + x.depth * W + w];
        }
    }
    if (moments && n_meas > 0)
        for (uint32_t u = threadIdx.x; u < nu; u += blockDim.x) {
            if (us[u].slab != 0) continue;
            double* mo = moments + 5 * (size_t)us[u].rep;
            if (ok && !aborted) store_moments(mo, n_meas, acc[u][0], acc[u][1], acc[u][2], acc[u][3], acc[u][4]);
            else for (int k = 0; k < 5; ++k) mo[k] = __builtin_nan("");
        }
}

// Unpack one replica's planes (L x L, the packed layout above) to int8 rows.
__global__ void k_batch_unpack(const BatchReplica* table, const uint32_t* state, uint32_t j, int8_t* spins) {
    const BatchReplica rp = table[j];
    const uint32_t L = rp.L, W = rp.W, words = L * W;
    const uint32_t* p = state + rp.state_off;
    for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < words; w += gridDim.x * blockDim.x) {
        const uint32_t r = w / W, g = w % W;
        const uint32_t q0 = p[w], q1 = p[words + w];
        const uint32_t even = (r & 1u) ? q1 : q0, odd = (r & 1u) ? q0 : q1;
        const uint32_t ncol = L >= 64 ? 64u : 32u;
        for (uint32_t d = 0; d < ncol / 4; ++d) {
            const uint32_t k = d >> 1, h = d & 1u, sh = 15 - k - 8 * h;
            const uint32_t v = perm(odd << sh, even << sh, 0x0B090A08u) | 0x01010101u;
            *reinterpret_cast<uint32_t*>(spins + (size_t)r * L + (size_t)g * 64u + 4u * d) = v;
        }
    }
}

// FP64 moments of a traced chain, summed in sweep order by one lane so the result does not
// depend on scheduling: out = (<|m|>, <m^2>, <m^4>, <e>, <e^2>) with m = M / N, e = E / N.
__global__ void k_moments(const int64_t* trace, int64_t n, int64_t n_sites, double* out) {
#pragma clang fp contract(off)
    // separate divides, multiplies and adds (no fused multiply-add), each rounded as written
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double N = (double)n_sites;
    double s_abs = 0.0, s_m2 = 0.0, s_m4 = 0.0, s_e = 0.0, s_e2 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double m = (double)trace[2 * i] / N, e = (double)trace[2 * i + 1] / N;
        const double m2 = m * m;
        s_abs += fabs(m);
        s_m2 += m2;
        s_m4 += m2 * m2;
        s_e += e;
        s_e2 += e * e;
    }
    const double k = (double)n;
    out[0] = s_abs / k;
    out[1] = s_m2 / k;
    out[2] = s_m4 / k;
    out[3] = s_e / k;
    out[4] = s_e2 / k;
}

// The device memory of ising_sweep_fused_static, for callers that cannot allocate: 64 MiB for the
// second lattice buffer (L <= 8192), then 512 KiB for the spread sets of its traced launches (64
// sets of 8 KiB).  Each GPU the library runs on holds its own copy from the module's load to the end
// of the process.
constexpr size_t kStaticLatticeBytes = size_t(64) << 20;
constexpr uint32_t kSpreadFold = 64;  // traced launches per fold (k_fold_spread)
constexpr size_t kSpreadBytes = size_t(kSpreadFold) * kSpreadSetWords * sizeof(int64_t);
constexpr size_t kStaticScratchBytes = kStaticLatticeBytes + kSpreadBytes;
__device__ __align__(256) int8_t scratch[kStaticScratchBytes];

}  // namespace ising

// ==========================================================================================
// Host side: validation, thresholds, launches.
namespace {

thread_local std::string g_last_error;

// Launch-shape options (ising_set_option).  Every valid setting gives bit-identical results.  Each
// one is an atomic, so a setting made on one thread while another launches is race-free (the launch
// sees the old or the new value, with the same results).
struct Options {
    std::atomic<int64_t> rows_per_lane = 0;  // 0 = choose from L
    std::atomic<int64_t> xcd_remap = 1;
    std::atomic<int64_t> nt_store = 0;
    std::atomic<int64_t> staged = 1;
    std::atomic<int64_t> batch_threads = 0;  // 0 = autotune
    std::atomic<int64_t> batch_slab_sites = 0;  // batch: split replicas into slabs of at most this many sites;
                                   // 0 = autotune, -1 = never split
    std::atomic<int64_t> batch_depth = 0;       // batch: colour updates between exchanges of split replicas; 0 = autotune
    std::atomic<int64_t> batch_lists_per_cu = 0;  // batch: work lists per compute unit of a split schedule; 0 = autotune
    std::atomic<int64_t> fused_rows = 0;     // rows per strip of the fused sweep; 0 = choose from L
    std::atomic<int64_t> fused_alternate = 1;  // fused sweep: odd strips walk upwards
    std::atomic<int64_t> fused_sweeps = 2;     // fused sweep: sweeps per pass over the lattice (1 or 2)
    std::atomic<int64_t> fused_ties = 1;       // two-sweep pass: settle the ties of a step's four updates together
    std::atomic<int64_t> fused_pairs = 1;      // two-sweep pass, rows of at most 512 groups: ties of two steps together
    std::atomic<int64_t> fused_bands = 0;      // two-sweep pass in column bands of one wave: 0 = above L = 16384, 1 = from 4096, 2 = above 65536
    std::atomic<int64_t> band_rows = 0;        // rows per strip of the band pass; 0 = choose from L
    std::atomic<int64_t> packed_ties = 1;      // packed half-sweep: settle the ties of four rows together
    std::atomic<int64_t> ties3 = 1;            // 3-D int8 half-sweep: two planes per exchange, ties settled together
    std::atomic<int64_t> planes3 = 0;          // 3-D sweep: planes per workgroup; 0 = choose from L
};
Options g_opt;

int hip_failed(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return ISING_EHIP;
}

int check_launch(const char* what) {
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? ISING_OK : hip_failed(e, what);
}

// square lattices: L a multiple of 32 (an odd multiple ends every row in a half group), 32 .. 2^20
bool valid_L(int64_t L) { return L >= 32 && L % 32 == 0 && L <= (int64_t(1) << 20); }

bool valid_beta(double beta) { return !std::isnan(beta) && beta >= 0.0; }

// Blocks of 256 threads for a grid-stride loop over n items: a dispatch holds fewer than 2^32
// work-items, and a million threads keep every compute unit busy.
unsigned grid_blocks(uint64_t n) { return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, 4096)); }

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

void host_thresholds(double beta, uint64_t T[2]) {
    for (int k = 0; k < 2; ++k) {
        const double s = k == 0 ? 2.0 : 4.0;
        double y = std::ceil(std::ldexp(std::exp(-2.0 * beta * s), 32));
        if (y > 4294967296.0) y = 4294967296.0;
        if (!(y >= 0.0)) y = 0.0;
        T[k] = (uint64_t)y;
    }
}

// ---- Low-precision acceptance (fmt 1 = bfloat16, 2 = IEEE half).  The probability is
// exp(-2 beta s) rounded to nearest-even in the format; the site's uniform is the top 16 bits
// r of its exact-chain uniform x, as r / 2^16 rounded toward zero in the format.  Rounding r / 2^16
// toward zero keeps the leading `digits` significant bits of r (no subnormal case arises: r / 2^16
// >= 2^-16 is normal in bfloat16, and below 2^-14 the half quantum 2^-24 is finer than 2^-16), so
// u(r) < p  <=>  r < R, R = the least r with trunc(r) >= p 2^16, and the acceptance becomes the
// exact-chain test x < R 2^16.
int fmt_digits(int fmt) { return fmt == 1 ? 8 : 11; }

// nearest-even rounding of p in [0, 1] to `digits` significant bits; half-precision values below
// 2^-14 are multiples of 2^-24, bfloat16 values below 2^-126 multiples of 2^-133.
double round_nearest_even(double p, int fmt) {
    if (!(p > 0.0)) return 0.0;
    const int digits = fmt_digits(fmt);
    const int min_normal_exp = fmt == 1 ? -126 : -14;
    if (p < std::ldexp(1.0, min_normal_exp)) {
        const double q = std::ldexp(1.0, min_normal_exp - digits + 1);
        return std::nearbyint(p / q) * q;
    }
    uint64_t bits;
    std::memcpy(&bits, &p, sizeof bits);
    const int drop = 52 - (digits - 1);                      // mantissa bits to clear
    const uint64_t half = uint64_t(1) << (drop - 1);
    const uint64_t lsb = (bits >> drop) & 1u;
    bits += half - 1 + lsb;                                  // ties go to the even neighbour
    bits &= ~((uint64_t(1) << drop) - 1);
    double r;
    std::memcpy(&r, &bits, sizeof r);
    return r;
}

uint32_t keep_leading_bits(uint32_t r, int digits) {
    if (r == 0) return 0;
    const int len = 32 - __builtin_clz(r);
    return len <= digits ? r : r & ~((1u << (len - digits)) - 1u);
}

void host_thresholds_fmt(double beta, int fmt, uint64_t T[2]) {
    if (fmt == 0) {
        host_thresholds(beta, T);
        return;
    }
    for (int k = 0; k < 2; ++k) {
        const double s = k == 0 ? 2.0 : 4.0;
        const double p16 = round_nearest_even(std::exp(-2.0 * beta * s), fmt) * 65536.0;
        uint32_t R = 65536;
        for (uint32_t r = 0; r < 65536; ++r)
            if ((double)keep_leading_bits(r, fmt_digits(fmt)) >= p16) { R = r; break; }
        T[k] = (uint64_t)R << 16;
    }
}

ising::Thresholds make_thresholds(double beta, int fmt = 0) {
    uint64_t T[2];
    host_thresholds_fmt(beta, fmt, T);
    ising::Thresholds th;
    const bool full2 = T[0] >= (uint64_t(1) << 32), full4 = T[1] >= (uint64_t(1) << 32);
    th.f2 = full2 ? 0xFFFFFFFFu : 0u;
    th.f4 = full4 ? 0xFFFFFFFFu : 0u;
    th.t2 = full2 ? 0u : (uint32_t)T[0];
    th.t4 = full4 ? 0u : (uint32_t)T[1];
    th.blocks = ((th.t2 | th.t4) & 0xFFFFu) == 0 ? 4u : 8u;
    return th;
}

// Column groups of a row: 64 columns each, the last one a half group of 32 when L is an odd multiple
// of 32.
uint32_t groups_of(int64_t L) { return (uint32_t)((L + 63) / 64); }

// rows per lane for the streaming kernels: even, divides L (L % 32 == 0)
uint32_t device_cus();

uint32_t rows_per_lane(int64_t L) {
    if (g_opt.rows_per_lane > 0 && L % g_opt.rows_per_lane == 0) return (uint32_t)g_opt.rows_per_lane;
    const uint32_t groups = groups_of(L);
    // tall strips re-read fewer boundary rows: the tallest up to 32 that keeps two waves per SIMD
    // (measured against four waves per SIMD: L = 8192 +25% at 8 rows, 16384 +2% at 32, 65536 and up
    // unchanged at 32; one wave per SIMD ran slower at 8192 and faster by 3% at 16384)
    const uint64_t min_lanes = (uint64_t)device_cus() * 4u * 2u * 64u;
    uint32_t R = 32;
    while (R > 2 && ((uint64_t)groups * (uint64_t)(L / R) < min_lanes || L % R != 0)) R >>= 1;
    return R;
}

int launch_half_sweep(int8_t* spins, int64_t L, const ising::Thresholds& th, uint64_t seed, uint32_t t,
                      int q, int64_t* obs, hipStream_t stream) {
    ising::SweepArgs a;
    a.spins = spins;
    a.L = (uint32_t)L;
    a.groups = groups_of(L);
    a.rows = rows_per_lane(L);
    a.n_lanes = a.groups * (uint32_t)(L / a.rows);
    a.t = t;
    a.key0 = (uint32_t)seed;
    a.key1 = (uint32_t)(seed >> 32);
    a.th = th;
    a.obs = obs;
    a.xcd_remap = g_opt.xcd_remap ? 1u : 0u;
    a.nt_store = g_opt.nt_store ? 1u : 0u;
    const dim3 grid((a.n_lanes + 255u) / 256u), block(256);
    // coalesced LDS-staged row I/O needs whole waves on 64 consecutive whole groups of one row
    const bool half = L % 64 != 0;
    const bool staged = g_opt.staged && a.groups % 64u == 0 && !half;
#define ISING_LAUNCH_SWEEP(QQ, OO, SS, HH) \
    hipLaunchKernelGGL((ising::k_sweep_int8<QQ, OO, SS, HH>), grid, block, 0, stream, a)
    if (half) {
        if (q == 1) { if (obs) ISING_LAUNCH_SWEEP(1, true, false, true); else ISING_LAUNCH_SWEEP(1, false, false, true); }
        else { if (obs) ISING_LAUNCH_SWEEP(0, true, false, true); else ISING_LAUNCH_SWEEP(0, false, false, true); }
    } else if (q == 1) {
        if (staged) { if (obs) ISING_LAUNCH_SWEEP(1, true, true, false); else ISING_LAUNCH_SWEEP(1, false, true, false); }
        else { if (obs) ISING_LAUNCH_SWEEP(1, true, false, false); else ISING_LAUNCH_SWEEP(1, false, false, false); }
    } else {
        if (staged) { if (obs) ISING_LAUNCH_SWEEP(0, true, true, false); else ISING_LAUNCH_SWEEP(0, false, true, false); }
        else { if (obs) ISING_LAUNCH_SWEEP(0, true, false, false); else ISING_LAUNCH_SWEEP(0, false, false, false); }
    }
#undef ISING_LAUNCH_SWEEP
    return check_launch("k_sweep_int8");
}

// The fused sweep puts a whole row in one workgroup (one thread per 64-column group).
constexpr int64_t kFusedMaxL = 64 * 1024;

// Rows per strip of a fused pass (even, divides L): the tallest (fewest re-read and recomputed rows
// around each strip) that still leaves 4096 waves, 8 at least; a two-sweep pass recomputes four rows
// on either side, so it starts from taller strips (128 against 64).
uint32_t fused_rows(int64_t L, int sweeps = 1) {
    if (g_opt.fused_rows > 0 && L % g_opt.fused_rows == 0 && g_opt.fused_rows <= L) return (uint32_t)g_opt.fused_rows;
    const uint64_t waves = (uint64_t)(L / 64 + 63) / 64;
    uint32_t R = sweeps == 2 ? 128 : 64;
    // R must divide L (64 always does): L = 64 (2k + 1) takes at most 64 rows
    while (R > 8 && ((uint64_t)(L / R) * waves < 4096ull || L % R != 0)) R >>= 1;
    return R;
}

// Compute units of the current device (cached per device).
uint32_t device_cus() {
    static std::atomic<uint32_t> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    uint32_t v = cache[dev].load(std::memory_order_relaxed);
    if (v == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        v = (uint32_t)n;
        cache[dev].store(v, std::memory_order_relaxed);
    }
    return v;
}

// Strips of the two-sweep pass with paired steps: S strips of R or R + 2 rows (R even), `tall` of them
// the taller.  Its waves hold up to 168 registers, three per SIMD: by default there are as many strips
// as the device holds at once (tall strips recompute fewer rows), of 8 to 128 rows; option fused_rows
// asks for strips of about that many rows.
struct PairStrips {
    uint32_t S, R, tall;
};

PairStrips fused_strips_pairs(int64_t L) {
    uint64_t S;
    if (g_opt.fused_rows > 0 && g_opt.fused_rows <= L) {
        S = ((uint64_t)L + (uint64_t)g_opt.fused_rows - 1) / (uint64_t)g_opt.fused_rows;
    } else {
        const uint64_t waves_per_strip = (uint64_t)(L / 64 + 63) / 64;
        const uint64_t slots = (uint64_t)device_cus() * 4u * 3u;
        S = std::max<uint64_t>(1, slots / waves_per_strip);
        S = std::min<uint64_t>(S, (uint64_t)L / 8);                 // 8 rows at least
        S = std::max<uint64_t>(S, ((uint64_t)L + 127) / 128);       // 128 rows at most
    }
    const uint64_t R = 2 * ((uint64_t)L / (2 * S));  // even; L - S R < 2 S
    return PairStrips{(uint32_t)S, (uint32_t)R, (uint32_t)(((uint64_t)L - S * R) / 2)};
}

// One pass of the fused kernel: `sweeps` (1 or 2) sweeps t, t + 1 from src to dst; obs: NULL or
// 2 * sweeps int64, zeroed beforehand, or with `spread` a spread set (zeroed beforehand).
int launch_fused_sweep(const int8_t* src, int8_t* dst, int64_t L, const ising::Thresholds& th, uint64_t seed,
                       uint32_t t, int64_t* obs, hipStream_t stream, int sweeps = 1, bool spread = false) {
    ising::FusedArgs a;
    a.src = src;
    a.dst = dst;
    a.L = (uint32_t)L;
    a.groups = (uint32_t)(L / 64);
    // paired steps: two sweeps with the ties of two steps settled together, rows of at most 512 groups
    const bool pairs = sweeps == 2 && g_opt.fused_ties != 0 && g_opt.fused_pairs != 0 && a.groups <= 512u;
    uint32_t n_strips;
    if (pairs) {
        const PairStrips ps = fused_strips_pairs(L);
        a.rows = ps.R;
        a.tall = ps.tall;
        n_strips = ps.S;
    } else {
        a.rows = fused_rows(L, sweeps);
        a.tall = 0;
        n_strips = a.L / a.rows;
    }
    a.t = t;
    a.key0 = (uint32_t)seed;
    a.key1 = (uint32_t)(seed >> 32);
    a.th = th;
    a.obs = obs;
    a.xcd_remap = g_opt.xcd_remap ? 1u : 0u;
    a.nt_store = g_opt.nt_store ? 1u : 0u;
    a.alternate = g_opt.fused_alternate ? 1u : 0u;
    // a kernel other than k_sweep_fused2q adds into the set's first line, which the fold counts as well
    a.spread = spread ? 1u : 0u;
    const uint32_t threads = (a.groups + 63u) / 64u * 64u;
    const bool staged = g_opt.staged && a.groups % 64u == 0;
    const bool ties = g_opt.fused_ties != 0;
    const size_t per_wave = pairs ? ising::kPairWaveBytes : ties ? ising::kTieQueueBytes : staged ? 4096u : 0u;
    const size_t lds = (size_t)(threads / 64u) * per_wave + 2u * threads * sizeof(uint32_t);
    const dim3 grid(n_strips), block(threads);
#define ISING_LAUNCH_FUSED(K, OO, SS)                                                                    \
    do {                                                                                                 \
        if (lds > 65536) {                                                                               \
            const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&ising::K<OO, SS>),   \
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
            if (e != hipSuccess) return hip_failed(e, "hipFuncSetAttribute(" #K ")");                   \
        }                                                                                                \
        hipLaunchKernelGGL((ising::K<OO, SS>), grid, block, lds, stream, a);                            \
    } while (0)
    if (pairs) {
        if (staged) { if (obs) ISING_LAUNCH_FUSED(k_sweep_fused2p, true, true); else ISING_LAUNCH_FUSED(k_sweep_fused2p, false, true); }
        else { if (obs) ISING_LAUNCH_FUSED(k_sweep_fused2p, true, false); else ISING_LAUNCH_FUSED(k_sweep_fused2p, false, false); }
        return check_launch("k_sweep_fused2p");
    }
    if (ties && sweeps == 2) {
        if (staged) { if (obs) ISING_LAUNCH_FUSED(k_sweep_fused2q, true, true); else ISING_LAUNCH_FUSED(k_sweep_fused2q, false, true); }
        else { if (obs) ISING_LAUNCH_FUSED(k_sweep_fused2q, true, false); else ISING_LAUNCH_FUSED(k_sweep_fused2q, false, false); }
        return check_launch("k_sweep_fused2q");
    }
    if (ties) {
        if (staged) { if (obs) ISING_LAUNCH_FUSED(k_sweep_fusedq, true, true); else ISING_LAUNCH_FUSED(k_sweep_fusedq, false, true); }
        else { if (obs) ISING_LAUNCH_FUSED(k_sweep_fusedq, true, false); else ISING_LAUNCH_FUSED(k_sweep_fusedq, false, false); }
        return check_launch("k_sweep_fusedq");
    }
    if (sweeps == 2) {
        if (staged) { if (obs) ISING_LAUNCH_FUSED(k_sweep_fused2, true, true); else ISING_LAUNCH_FUSED(k_sweep_fused2, false, true); }
        else { if (obs) ISING_LAUNCH_FUSED(k_sweep_fused2, true, false); else ISING_LAUNCH_FUSED(k_sweep_fused2, false, false); }
        return check_launch("k_sweep_fused2");
    }
    if (staged) { if (obs) ISING_LAUNCH_FUSED(k_sweep_fused, true, true); else ISING_LAUNCH_FUSED(k_sweep_fused, false, true); }
    else { if (obs) ISING_LAUNCH_FUSED(k_sweep_fused, true, false); else ISING_LAUNCH_FUSED(k_sweep_fused, false, false); }
#undef ISING_LAUNCH_FUSED
    return check_launch("k_sweep_fused");
}

// The two-sweep pass runs in column bands above kBandsAboveL by default (above kFusedMaxL always).
// Between the two the row kernels were measured 6-75% slower than the bands (at L = 20480 ... 65536),
// and at L = 16384 14% faster.  Option "fused_bands": 1 = bands from L = 4096 (a band's 64 lanes then
// take 64 distinct groups), 2 = rows wherever a whole row fits a workgroup.
constexpr int64_t kBandsAboveL = 16384;
bool use_bands(int64_t L) {
    if (L > kFusedMaxL) return true;
    if (g_opt.fused_bands == 1) return L >= 4096;
    return g_opt.fused_bands == 0 && L > kBandsAboveL;
}

// Bands per row: each owns at most 62 groups (its wave has one recomputed group on either side).
uint32_t band_count(int64_t L) { return (uint32_t)((L / 64 + 61) / 62); }

// Rows per strip of the band pass: the power of two in [8, 256] dividing L whose launch costs least
// under a count of the waves each SIMD runs.  A strip of R rows costs R + 10 rows of work (the
// recomputed halo rows of the two sweeps); a launch of W waves puts ceil(W / SIMDs) of them on the
// busiest SIMD, and a SIMD that holds a single wave has no other wave to cover its latency and runs
// it at about half speed.  The smallest cost picked the fastest of 8 ... 256 rows, or one within
// 0.7% of it, at every L measured (16384 ... 65536 and 131072: 32 rows at 16384, 64 or 128 between,
// 256 at 131072).
uint32_t band_rows(int64_t L) {
    if (g_opt.band_rows > 0 && L % g_opt.band_rows == 0 && g_opt.band_rows <= L) return (uint32_t)g_opt.band_rows;
    const uint64_t bands = band_count(L), simds = (uint64_t)device_cus() * 4u;
    uint32_t best = 8;
    uint64_t best_cost = UINT64_MAX;
    for (uint32_t R = 8; R <= 256 && R <= L; R <<= 1) {
        if (L % R != 0) continue;
        const uint64_t waves = bands * (uint64_t)(L / R), per_simd = (waves + simds - 1) / simds;
        const uint64_t cost = (per_simd == 1 ? 2u : per_simd) * (R + 10u);
        if (cost < best_cost) best = R, best_cost = cost;  // ties keep the shorter strip
    }
    return best;
}

// One two-sweep pass in column bands: sweeps t, t + 1 from src to dst; obs: NULL or 4 int64, zeroed
// beforehand.
int launch_band_pass(const int8_t* src, int8_t* dst, int64_t L, const ising::Thresholds& th, uint64_t seed,
                     uint32_t t, int64_t* obs, hipStream_t stream) {
    ising::BandArgs a;
    a.src = src;
    a.dst = dst;
    a.L = (uint32_t)L;
    a.groups = (uint32_t)(L / 64);
    a.rows = band_rows(L);
    a.bands = band_count(L);
    a.units = a.bands * (a.L / a.rows);
    a.t = t;
    a.key0 = (uint32_t)seed;
    a.key1 = (uint32_t)(seed >> 32);
    a.th = th;
    a.obs = obs;
    a.xcd_remap = g_opt.xcd_remap ? 1u : 0u;
    a.nt_store = g_opt.nt_store ? 1u : 0u;
    a.alternate = g_opt.fused_alternate ? 1u : 0u;
    constexpr uint32_t waves = 4;
    const dim3 grid((a.units + waves - 1) / waves), block(64 * waves);
    if (g_opt.fused_ties != 0 && g_opt.fused_pairs != 0) {
        // the paired walk: two steps per settle
        const size_t lds = waves * ising::kPairWaveBytes;
        if (obs) hipLaunchKernelGGL((ising::k_sweep_fused2pb<true>), grid, block, lds, stream, a);
        else hipLaunchKernelGGL((ising::k_sweep_fused2pb<false>), grid, block, lds, stream, a);
        return check_launch("k_sweep_fused2pb");
    }
    const size_t lds = waves * ising::kTieQueueBytes;
    if (obs) hipLaunchKernelGGL((ising::k_sweep_fused2b<true>), grid, block, lds, stream, a);
    else hipLaunchKernelGGL((ising::k_sweep_fused2b<false>), grid, block, lds, stream, a);
    return check_launch("k_sweep_fused2b");
}

bool disjoint(const void* a, const void* b, uint64_t bytes) {
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x + bytes <= y || y + bytes <= x;
}

bool disjoint_ranges(const void* a, uint64_t a_bytes, const void* b, uint64_t b_bytes) {
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x + a_bytes <= y || y + b_bytes <= x;
}

int zero_trace(int64_t* p, int64_t n, hipStream_t stream) {
    if (n <= 0) return ISING_OK;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(ising::k_zero_n, dim3((unsigned)blocks), dim3(256), 0, stream, p, n);
    return check_launch("k_zero_n");
}

// The device address of ising::scratch on the current device, looked up once per device (with that
// device current) and kept: in host code the array's name is only a host-side stand-in.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int8_t* g_scratch_addr[kMaxDevices] = {};

int static_scratch(int8_t** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_failed(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return ISING_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(ising::scratch));
        if (e != hipSuccess) return hip_failed(e, "hipGetSymbolAddress(scratch)");
        g_scratch_addr[dev] = reinterpret_cast<int8_t*>(p);
    }
    *out = g_scratch_addr[dev];
    return ISING_OK;
}

// ---- Spread sets of the traced sweep loops.  Up to kSpreadFold traced launches take a set each
// (their workgroups add (M, E) into the set's lines, see spread_line), then one k_fold_spread launch
// writes each set's sums into its trace entries and clears the set.  The sets come from a
// stream-ordered pool that the library keeps per device, so that calls on different streams never
// share one and no call waits for another; ising_sweep_fused_static passes its own.
std::mutex g_pool_mu;
hipMemPool_t g_pool[kMaxDevices] = {};

int spread_pool(hipMemPool_t* out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_failed(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return ISING_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_pool_mu);
    if (!g_pool[dev]) {
        hipMemPoolProps props = {};
        props.allocType = hipMemAllocationTypePinned;
        props.handleTypes = hipMemHandleTypeNone;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = dev;
        hipMemPool_t pool = nullptr;
        e = hipMemPoolCreate(&pool, &props);
        if (e != hipSuccess) return hip_failed(e, "hipMemPoolCreate");
        // keep freed blocks for the next calls rather than returning them at each synchronisation
        uint64_t keep = UINT64_MAX;
        e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
        if (e != hipSuccess) {
            (void)hipMemPoolDestroy(pool);
            return hip_failed(e, "hipMemPoolSetAttribute");
        }
        g_pool[dev] = pool;
    }
    *out = g_pool[dev];
    return ISING_OK;
}

using ising_host::SpreadTrace;

}  // namespace

// ---- batched replicas --------------------------------------------------------------------------
namespace {

constexpr size_t kTableAlign = 256;
// dynamic LDS of a work list that leaves room for at most `per_cu` workgroups on a compute unit
// (160 KiB of LDS; the kernel's static LDS adds about 5 KiB)
size_t lds_floor(int per_cu) { return per_cu == 1 ? 81920 : 55296; }
size_t lds_cap(int per_cu) { return per_cu == 1 ? 131072 : 73728; }

size_t align_up(size_t x) { return (x + kTableAlign - 1) / kTableAlign * kTableAlign; }

// 32 (one 16-site word per row and colour) or a multiple of 64 (whole 32-site words), at most 512
bool valid_batch_L(int64_t L) { return L == 32 || (L >= 64 && L <= 512 && L % 64 == 0); }

uint32_t batch_W(int64_t L) { return L >= 64 ? (uint32_t)(L / 64) : 1u; }

uint64_t batch_words(int64_t L) { return 2ull * (uint64_t)L * batch_W(L); }

// Workspace: replica table | per-call values | both colour planes of every replica | work lists |
// units | exchange areas.
struct BatchLayout {
    size_t params, state, groups, units, exchange, total;
};

size_t batch_params_offset(int64_t n) { return align_up((size_t)n * sizeof(ising::BatchReplica)); }
size_t batch_state_offset(int64_t n) { return align_up(batch_params_offset(n) + sizeof(ising::BatchRun)); }

BatchLayout batch_layout(const ising_replica_t* reps, int64_t n) {
    BatchLayout b{};
    b.params = batch_params_offset(n);
    b.state = batch_state_offset(n);
    uint64_t words = 0, xwords = 0;
    for (int64_t i = 0; i < n; ++i) {
        words += batch_words(reps[i].L);
        xwords += ising::exchange_words(batch_W(reps[i].L));
    }
    b.groups = align_up(b.state + words * 4u);
    b.units = align_up(b.groups + (size_t)n * ising::kMaxSlabs * sizeof(ising::BatchGroup));
    b.exchange = align_up(b.units + (size_t)n * ising::kMaxSlabs * sizeof(ising::BatchUnit));
    b.total = b.exchange + xwords * 8u;
    return b;
}

// Slabs of replica L for a split target (sites per slab; <= 0: one slab): halve the rows while
// the slab holds more than `target` sites, keeping at least 16 rows and at most kMaxSlabs slabs.
uint32_t slabs_for(int64_t L, int64_t target) {
    uint32_t P = 1;
    if (target <= 0 || L < 64) return 1;
    while (P < ising::kMaxSlabs && L * L / P > target && L % (2 * P) == 0 && L / (2 * P) >= 16) P *= 2;
    return P;
}

// Work lists of a schedule.  Unsplit: one replica per workgroup.  Split: the units (slabs and
// whole replicas) are packed into `per_cu` workgroups per compute unit, largest first onto the
// least loaded list, and each workgroup asks for enough LDS that no more than `per_cu` share a
// compute unit -- every workgroup is then resident at once, which the slabs' waits for their
// neighbours need.
struct BatchPlan {
    std::vector<ising::BatchGroup> groups;
    std::vector<ising::BatchUnit> units;   // in work-list order
    size_t lds = 0;                        // dynamic LDS bytes per workgroup
    uint32_t depth = 0;                    // colour updates between exchanges (0: nothing split)
    int per_cu = 1;                        // workgroups per compute unit (split plans)
    bool ok = false;
};

BatchPlan plan_batch(const ising_replica_t* reps, int64_t n, int64_t target, uint32_t depth, int per_cu, int cus) {
    BatchPlan plan;
    std::vector<ising::BatchUnit> all;
    std::vector<uint32_t> cost;
    uint64_t xoff = 0;
    bool split = false;
    for (int64_t i = 0; i < n; ++i) {
        const uint32_t P = slabs_for(reps[i].L, target), rows = (uint32_t)reps[i].L / P, W = batch_W(reps[i].L);
        const uint32_t K = P > 1 ? depth : 0u;
        for (uint32_t p = 0; p < P; ++p) {
            ising::BatchUnit x{};
            x.rep = (uint32_t)i;
            x.slab = p;
            x.slabs = P;
            x.row0 = p * rows;
            x.rows = rows;
            x.depth = K;
            // a slab starts exchange period e + 1 only after its neighbours finished period e, so
            // one d slabs away has finished at least (d + 1) K colour updates fewer: the counts
            // of sweep j are all in place (P / 2 + 1) K / 2 sweeps later
            x.lag = ((P / 2 + 1) * K + 1) / 2;
            x.xoff = xoff;
            all.push_back(x);
            cost.push_back((ising::unit_words(rows, K, W) + 63u) / 64u * 64u + 64u);
        }
        split = split || P > 1;
        xoff += ising::exchange_words(W);
    }
    std::vector<std::vector<uint32_t>> lists;
    if (!split) {
        for (uint32_t k = 0; k < all.size(); ++k) lists.push_back({k});
    } else {
        const size_t G = std::min<size_t>(all.size(), (size_t)std::max(cus, 1) * (size_t)per_cu);
        lists.resize(G);
        std::vector<uint32_t> order(all.size());
        for (uint32_t k = 0; k < order.size(); ++k) order[k] = k;
        std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return cost[a] > cost[b]; });
        using Load = std::pair<uint64_t, uint32_t>;
        std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
        for (uint32_t g = 0; g < G; ++g) heap.push({0, g});
        for (uint32_t k : order) {
            Load top = heap.top();
            heap.pop();
            lists[top.second].push_back(k);
            top.first += cost[k];
            heap.push(top);
        }
    }
    size_t lds_max = 0;
    for (const auto& list : lists) {
        if (list.empty()) continue;
        if (list.size() > ising::kMaxUnits) return plan;
        ising::BatchGroup grp{};
        grp.begin = (uint32_t)plan.units.size();
        uint32_t lds = 0, first = 0, xfirst = 0;
        for (uint32_t k : list) {
            ising::BatchUnit x = all[k];
            const uint32_t W = batch_W(reps[x.rep].L);
            x.lds = lds;
            x.first = first;
            x.xfirst = xfirst;
            lds += 2u * ising::unit_plane(x.rows, x.depth, W);
            first += (ising::unit_words(x.rows, x.depth, W) + 63u) / 64u;   // whole waves
            xfirst += x.depth ? ising::unit_xwords(x.depth, W) : 0u;
            plan.units.push_back(x);
        }
        grp.end = (uint32_t)plan.units.size();
        grp.words = first;
        grp.xwords = xfirst;
        plan.groups.push_back(grp);
        lds_max = std::max(lds_max, (size_t)lds * 4u);
    }
    if (split && lds_max > lds_cap(per_cu)) return plan;
    plan.lds = split ? std::max(lds_max, lds_floor(per_cu)) : lds_max;
    plan.per_cu = per_cu;
    plan.depth = split ? depth : 0u;
    plan.ok = true;
    return plan;
}

// Captured batch runs, one per plan (workspace address, layout and schedule; the per-call values
// live in the workspace), least recently used dropped first.  Guarded by g_batch_mu, which every
// batch entry point holds for its whole call (the tuned schedules below too).
struct BatchExec {
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;  // recorded after the exec's latest launch
    uint64_t used = 0;
};
constexpr size_t kMaxBatchExecs = 8;
std::map<std::string, BatchExec> g_batch_execs;
hipStream_t g_batch_capture = nullptr;
uint64_t g_batch_clock = 0;
std::mutex g_batch_mu;

struct BatchSchedule {
    int threads;
    int64_t target;  // split target (sites per slab), -1 = none
    int depth;       // colour updates between exchanges of a split replica
    int per_cu;      // work lists per compute unit of a split schedule
};
std::map<std::string, BatchSchedule> g_batch_tuned;  // replica-size signature -> schedule

std::string batch_signature(const ising_replica_t* reps, int64_t n) {
    std::string sig;
    for (int64_t i = 0; i < n; ++i) sig += std::to_string(reps[i].L) + ",";
    return sig;
}

int compute_units() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus;
}

// A split plan runs only if its workgroups can all be resident at once.
bool plan_fits(const BatchPlan& plan, int threads, int cus) {
    if (!plan.ok) return false;
    if (plan.depth == 0) return true;
    if (plan.lds > 65536) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&ising::k_batch),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)plan.lds);
        if (e != hipSuccess) return false;
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ising::k_batch, threads, plan.lds) != hipSuccess)
        return false;
    return per_cu >= plan.per_cu && (int64_t)plan.groups.size() <= (int64_t)cus * plan.per_cu;
}

struct BatchBuffers {
    ising::BatchRun* run;
    const ising::BatchReplica* table;
    ising::BatchGroup* groups;
    ising::BatchUnit* units;
    uint32_t* state;
    uint64_t* exchange;
    int64_t exchange_words;
};

// Copy a plan's tables into the workspace (the host vectors may be reused on return: a copy from
// pageable memory has read them by then).
int upload_plan(const BatchBuffers& b, const BatchPlan& plan, hipStream_t stream) {
    hipError_t e = hipMemcpyAsync(b.groups, plan.groups.data(), plan.groups.size() * sizeof(ising::BatchGroup),
                                  hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_failed(e, "hipMemcpyAsync(work lists)");
    e = hipMemcpyAsync(b.units, plan.units.data(), plan.units.size() * sizeof(ising::BatchUnit), hipMemcpyHostToDevice,
                       stream);
    if (e != hipSuccess) return hip_failed(e, "hipMemcpyAsync(units)");
    return ISING_OK;
}

// The per-call values of a run, written into the workspace on `stream` ahead of the run.
int set_batch_run(const BatchBuffers& b, uint32_t start, uint32_t n_therm, uint32_t n_meas, int64_t* trace,
                  double* moments, hipStream_t stream) {
    ising::BatchRun v{start, n_therm, n_meas, 0u, trace, moments};
    hipLaunchKernelGGL(ising::k_batch_set_run, dim3(1), dim3(64), 0, stream, b.run, v);
    return check_launch("k_batch_set_run");
}

// The exchange area is cleared by a kernel (tags start at 0 for every run), then the run.
int launch_batch(const BatchBuffers& b, const BatchPlan& plan, int threads, hipStream_t stream) {
    if (plan.depth > 0) {
        const int rc = zero_trace(reinterpret_cast<int64_t*>(b.exchange), b.exchange_words, stream);
        if (rc) return rc;
    }
    hipLaunchKernelGGL(ising::k_batch, dim3((unsigned)plan.groups.size()), dim3((unsigned)threads), plan.lds, stream,
                       b.table, b.groups, b.units, b.state, b.exchange, plan.depth, b.run);
    return check_launch("k_batch");
}

// Time each schedule on the replica table itself (thermalisation sweeps, which the real run
// overwrites) and keep the fastest; every schedule gives identical results.
int autotune_batch(const ising_replica_t* reps, int64_t n, const BatchBuffers& b, uint32_t start, hipStream_t stream,
                   BatchSchedule fixed, int cus, BatchSchedule* out) {
    const std::string sig = batch_signature(reps, n);
    auto it = g_batch_tuned.find(sig);
    if (it != g_batch_tuned.end()) { *out = it->second; return ISING_OK; }
    std::vector<BatchSchedule> cands;
    for (int64_t target : {int64_t(-1), int64_t(65536), int64_t(32768), int64_t(16384)}) {
        if (fixed.target && target != fixed.target) continue;
        for (int depth : {1, 2, 4}) {
            if (fixed.depth && depth != fixed.depth) continue;
            for (int per_cu : {1, 2}) {
                if (fixed.per_cu && per_cu != fixed.per_cu) continue;
                // depth and lists per CU only matter for split replicas
                if (target == -1 && (depth != (fixed.depth ? fixed.depth : 1) ||
                                     per_cu != (fixed.per_cu ? fixed.per_cu : 1)))
                    continue;
                for (int threads : {256, 512, 1024}) {
                    if (fixed.threads && threads != fixed.threads) continue;
                    if (target != -1 && threads == 256 && !fixed.threads) continue;   // few lists: wide groups
                    cands.push_back(BatchSchedule{threads, target, depth, per_cu});
                }
            }
        }
    }
    if (fixed.target > 0 && cands.empty()) cands.push_back(fixed);
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return hip_failed(e, "hipEventCreate");
    e = hipEventCreate(&e1);
    if (e != hipSuccess) { (void)hipEventDestroy(e0); return hip_failed(e, "hipEventCreate"); }
    BatchSchedule best{1024, -1, 1, 1};
    float best_ms = 1e30f;
    int rc = ISING_OK;
    for (const BatchSchedule& c : cands) {
        const BatchPlan plan = plan_batch(reps, n, c.target, (uint32_t)c.depth, c.per_cu, cus);
        if (!plan_fits(plan, c.threads, cus)) continue;
        rc = upload_plan(b, plan, stream);
        // the fastest of three 32-sweep runs, after one untimed run
        for (int rep = 0; rep < 4 && rc == ISING_OK; ++rep) {
            rc = set_batch_run(b, start, 32u, 0u, nullptr, nullptr, stream);
            if (rc) break;
            (void)hipEventRecord(e0, stream);
            rc = launch_batch(b, plan, c.threads, stream);
            (void)hipEventRecord(e1, stream);
            if (rc) break;
            e = hipEventSynchronize(e1);
            if (e != hipSuccess) { rc = hip_failed(e, "hipEventSynchronize"); break; }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (rep > 0 && ms < best_ms) { best_ms = ms; best = c; }
        }
        if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    g_batch_tuned[sig] = best;
    *out = best;
    return ISING_OK;
}

}  // namespace

namespace {
// Rows per lane of the packed half-sweep: a lane's word is 32 sites (a quarter of the int8 lane's
// 128), so it takes more lanes to fill the chip.  The tallest strip up to 32 rows that leaves 2^18
// lanes (4 waves per SIMD), 4 rows at least (the tie queue takes four rows at a time).  At L = 16384,
// 16 rows ran 1.7% faster than 8 (with the falling issue priority) and 4 rows 3% slower.
uint32_t packed_rows(int64_t L) {
    if (g_opt.rows_per_lane > 0 && L % g_opt.rows_per_lane == 0) return (uint32_t)g_opt.rows_per_lane;
    const uint64_t groups = groups_of(L);
    uint32_t R = 32;
    while (R > 4 && (groups * (uint64_t)(L / R) < (1ull << 18) || L % R != 0)) R >>= 1;
    return R;
}

using PackedKernel = void (*)(ising::PackedArgs);

template <int Q, bool OBS>
PackedKernel pick_packed_q(bool half, bool o32, bool urow) {
    if (half) return o32 ? ising::k_sweep_packed_q<Q, OBS, true, true> : ising::k_sweep_packed_q<Q, OBS, true, false>;
    if (urow)
        return o32 ? ising::k_sweep_packed_q<Q, OBS, false, true, true> : ising::k_sweep_packed_q<Q, OBS, false, false, true>;
    return o32 ? ising::k_sweep_packed_q<Q, OBS, false, true> : ising::k_sweep_packed_q<Q, OBS, false, false>;
}

// Workgroups of a kernel resident per CU (0 when the query fails), cached per device, kernel and
// shape.
uint32_t blocks_per_cu(const void* kern, uint32_t threads, size_t lds) {
    static std::mutex mu;
    static std::map<std::tuple<int, const void*, uint32_t, size_t>, uint32_t> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    const auto key = std::make_tuple(dev, kern, threads, lds);
    std::lock_guard<std::mutex> lock(mu);
    const auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, (int)threads, lds) != hipSuccess || n < 0) n = 0;
    cache[key] = (uint32_t)n;
    return (uint32_t)n;
}

int launch_half_sweep_packed(uint32_t* planes, int64_t L, const ising::Thresholds& th, uint64_t seed, uint32_t t,
                             int q, int64_t* obs, hipStream_t stream) {
    ising::PackedArgs a;
    a.planes = planes;
    a.L = (uint32_t)L;
    a.groups = groups_of(L);
    a.rows = packed_rows(L);
    a.n_lanes = a.groups * (uint32_t)(L / a.rows);
    a.t = t;
    a.key0 = (uint32_t)seed;
    a.key1 = (uint32_t)(seed >> 32);
    a.th = th;
    a.obs = obs;
    a.xcd_remap = g_opt.xcd_remap ? 1u : 0u;
    a.falling_prio = 0u;
    const bool half = L % 64 != 0;  // each row ends in a half group
    const dim3 grid((a.n_lanes + 255u) / 256u), block(256);
#define ISING_LAUNCH_PACKED(K, QQ, OO, G, B, LDS)                                                  \
    do {                                                                                           \
        if (half) hipLaunchKernelGGL((ising::K<QQ, OO, true>), G, B, LDS, stream, a);              \
        else hipLaunchKernelGGL((ising::K<QQ, OO, false>), G, B, LDS, stream, a);                  \
    } while (0)
    if (g_opt.packed_ties && a.rows % 4u == 0) {
        // a counting launch takes 512 threads per workgroup (half the end-of-launch reductions of
        // 256; measured no slower), the others 256, which leaves more waves per CU
        const uint32_t threads = obs ? 512u : 256u;
        const dim3 qgrid((a.n_lanes + threads - 1u) / threads), qblock(threads);
        const size_t lds = (threads / 64u) * ising::kTieQueueBytes;
        // 32-bit offsets within a plane while it spans at most 4 GiB (L <= 2^18)
        const bool o32 = (uint64_t)L * a.groups * 4u <= (uint64_t(1) << 32);
        // whole waves in one strip (64 whole groups per wave of a row)
        const bool urow = !half && a.groups % 64u == 0;
        PackedKernel kern = nullptr;
        if (q == 1) kern = obs ? pick_packed_q<1, true>(half, o32, urow) : pick_packed_q<1, false>(half, o32, urow);
        else kern = obs ? pick_packed_q<0, true>(half, o32, urow) : pick_packed_q<0, false>(half, o32, urow);
        // falling issue priority shortens the tail of a launch of one or two rounds of workgroups
        // (+2% at one round, +1.5% at 1.3 rounds); over many rounds it costs about 1%
        const uint32_t per_cu = blocks_per_cu(reinterpret_cast<const void*>(kern), threads, lds);
        a.falling_prio = per_cu > 0 && qgrid.x <= 2u * per_cu * device_cus() ? 1u : 0u;
        void* args[] = {&a};
        const hipError_t e = hipLaunchKernel(reinterpret_cast<const void*>(kern), qgrid, qblock, args, lds, stream);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return hip_failed(e, "k_sweep_packed_q");
        }
        return check_launch("k_sweep_packed_q");
    }
    if (q == 1) {
        if (obs) ISING_LAUNCH_PACKED(k_sweep_packed, 1, true, grid, block, 0);
        else ISING_LAUNCH_PACKED(k_sweep_packed, 1, false, grid, block, 0);
    } else {
        if (obs) ISING_LAUNCH_PACKED(k_sweep_packed, 0, true, grid, block, 0);
        else ISING_LAUNCH_PACKED(k_sweep_packed, 0, false, grid, block, 0);
    }
#undef ISING_LAUNCH_PACKED
    return check_launch("k_sweep_packed");
}
}  // namespace

namespace {

// n_sweeps sweeps in place, one launch per colour; trace_ME: NULL or 2 n_sweeps int64 (M, E after
// each sweep).  sets: kSpreadBytes for the spread sets of the traced launches, or NULL (the pool).
int sweep_int8(int8_t* spins, int64_t L, const ising::Thresholds& th, int64_t n_sweeps, uint64_t seed,
               uint64_t sweep_offset, int64_t* trace_ME, hipStream_t s, int64_t* sets) {
    SpreadTrace sp;
    if (trace_ME && n_sweeps > 0) {
        const int rc = sp.begin(sets, n_sweeps, s);
        if (rc) return rc;
    }
    for (int64_t i = 0; i < n_sweeps; ++i) {
        const uint32_t t = (uint32_t)(sweep_offset + (uint64_t)i);
        int64_t* set = nullptr;
        if (trace_ME) {
            const int rc = sp.next(trace_ME + 2 * i, 2, &set);
            if (rc) return rc;
        }
        int rc = launch_half_sweep(spins, L, th, seed, t, 1, nullptr, s);  // white
        if (rc) return rc;
        rc = launch_half_sweep(spins, L, th, seed, t, 0, set, s);          // black (+ M, E)
        if (rc) return rc;
    }
    return sp.fold();
}

// ising_sweep_fused after validation (scratch: the second lattice buffer; sets as in sweep_int8).
int sweep_fused(int8_t* spins, int8_t* scratch, int64_t L, const ising::Thresholds& th, int64_t n_sweeps,
                uint64_t seed, uint64_t sweep_offset, int64_t* trace_ME, hipStream_t s, int64_t* sets) {
    // the passes take whole 64-column groups: a row that ends in a half group sweeps in place
    if (L % 64 != 0) return sweep_int8(spins, L, th, n_sweeps, seed, sweep_offset, trace_ME, s, sets);
    const bool bands = use_bands(L);
    const bool single_passes = L <= kFusedMaxL;  // the one-sweep pass needs a whole row per workgroup
    const bool two = g_opt.fused_sweeps == 2;
    if (!single_passes && !two) return sweep_int8(spins, L, th, n_sweeps, seed, sweep_offset, trace_ME, s, sets);
    int64_t i = 0;
    if (n_sweeps & 1) {  // an odd count: the first sweep in place, so that the pairs end in `spins`
        const int rc = sweep_int8(spins, L, th, 1, seed, sweep_offset, trace_ME, s, sets);
        if (rc) return rc;
        i = 1;
    }
    if (trace_ME) {  // for the launches that add into the trace itself
        const int rc = zero_trace(trace_ME + 2 * i, 2 * (n_sweeps - i), s);
        if (rc) return rc;
    }
    // The rest (an even count) in passes that alternate between the two buffers and end in
    // `spins`: two sweeps per pass when the option allows, in an even number of passes.  An odd
    // number of two-sweep passes gives one of them up for two one-sweep passes, or, where there is no
    // one-sweep pass (above L = 65536), for two sweeps in place at the end.  Traced full-row
    // two-sweep passes add (M, E) into spread sets.
    const int64_t rest = n_sweeps - i;
    int64_t pairs = two ? rest / 2 : 0;
    if (pairs & 1) --pairs;
    SpreadTrace sp;
    if (trace_ME && pairs > 0 && !bands) {
        const int rc = sp.begin(sets, pairs, s);
        if (rc) return rc;
    }
    int8_t* bufs[2] = {spins, scratch};
    int64_t pass = 0;
    while (i < n_sweeps) {
        const uint32_t t = (uint32_t)(sweep_offset + (uint64_t)i);
        int64_t* obs = trace_ME ? trace_ME + 2 * i : nullptr;
        int rc = ISING_OK;
        if (pairs > 0) {
            if (bands) {
                rc = launch_band_pass(bufs[pass & 1], bufs[(pass + 1) & 1], L, th, seed, t, obs, s);
            } else {
                int64_t* set = nullptr;
                if (obs) rc = sp.next(obs, 4, &set);
                if (!rc)
                    rc = launch_fused_sweep(bufs[pass & 1], bufs[(pass + 1) & 1], L, th, seed, t, set ? set : obs, s, 2,
                                            set != nullptr);
            }
            --pairs;
            i += 2;
            ++pass;
        } else if (single_passes) {
            rc = launch_fused_sweep(bufs[pass & 1], bufs[(pass + 1) & 1], L, th, seed, t, obs, s, 1);
            i += 1;
            ++pass;
        } else {
            rc = sp.fold();  // the in-place sweeps may take the same sets
            if (!rc) rc = sweep_int8(spins, L, th, n_sweeps - i, seed, t, obs, s, sets);
            i = n_sweeps;
        }
        if (rc) return rc;
    }
    return sp.fold();
}

}  // namespace

// Definitions of the helpers declared in host.hpp (used by the 3-D translation unit).
namespace ising_host {
int hip_failed(hipError_t e, const char* what) { return ::hip_failed(e, what); }
int check_launch(const char* what) { return ::check_launch(what); }
bool valid_beta(double beta) { return ::valid_beta(beta); }
bool aligned16(const void* p) { return ::aligned16(p); }
bool xcd_remap() { return g_opt.xcd_remap != 0; }
int64_t option(const char* name) {
    int64_t v = 0;
    return ising_get_option(name, &v) == ISING_OK ? v : 0;
}
int zero_trace(int64_t* p, int64_t n, hipStream_t stream) { return ::zero_trace(p, n, stream); }

SpreadTrace::~SpreadTrace() {
    if (owned_) (void)hipFreeAsync(sets_, s_);
}

int SpreadTrace::begin(int64_t* given, int64_t n_launches, hipStream_t s) {
    s_ = s;
    if (given) {
        sets_ = given;
    } else {
        hipMemPool_t pool = nullptr;
        const int rc = spread_pool(&pool);
        if (rc) return rc;
        void* p = nullptr;
        const hipError_t e = hipMallocFromPoolAsync(&p, ising::kSpreadBytes, pool, s);
        if (e != hipSuccess) return hip_failed(e, "hipMallocFromPoolAsync");
        sets_ = static_cast<int64_t*>(p);
        owned_ = true;
    }
    const int64_t n = std::min<int64_t>(n_launches, ising::kSpreadFold);
    return zero_trace(sets_, n * (int64_t)ising::kSpreadSetWords, s);
}

int SpreadTrace::next(int64_t* dst, uint32_t n, int64_t** set) {
    if (used_ == ising::kSpreadFold || (used_ > 0 && (n != n_ || dst != dst0_ + (size_t)used_ * n_))) {
        const int rc = fold();
        if (rc) return rc;
    }
    if (used_ == 0) {
        dst0_ = dst;
        n_ = n;
    }
    *set = sets_ + (size_t)used_ * ising::kSpreadSetWords;
    ++used_;
    return ISING_OK;
}

int SpreadTrace::fold() {
    if (used_ == 0) return ISING_OK;
    hipLaunchKernelGGL(ising::k_fold_spread, dim3(used_), dim3(64), 0, s_, sets_, dst0_, n_);
    used_ = 0;
    return check_launch("k_fold_spread");
}
}  // namespace ising_host

extern "C" {

int ising_thresholds(double beta, uint64_t out[2]) {
    if (!out || !valid_beta(beta)) return ISING_EINVAL;
    host_thresholds(beta, out);
    return ISING_OK;
}

int ising_thresholds_fmt(double beta, int fmt, uint64_t out[2]) {
    if (!out || !valid_beta(beta) || fmt < 0 || fmt > 2) return ISING_EINVAL;
    host_thresholds_fmt(beta, fmt, out);
    return ISING_OK;
}

int ising_moments(const int64_t* trace_ME, int64_t n, int64_t n_sites, double* out, void* stream) {
    if (!trace_ME || !out || n <= 0 || n_sites <= 0) return ISING_EINVAL;
    hipLaunchKernelGGL(ising::k_moments, dim3(1), dim3(64), 0, (hipStream_t)stream, trace_ME, n, n_sites, out);
    return check_launch("k_moments");
}

int ising_init(int8_t* spins, int64_t L, uint64_t seed, void* stream) {
    if (!spins || !valid_L(L) || !aligned16(spins)) return ISING_EINVAL;
    const uint32_t chunks = (uint32_t)((L + 127) / 128);
    const uint64_t n_lanes = (uint64_t)chunks * (uint64_t)L;
    const dim3 grid(grid_blocks(n_lanes)), block(256);
    hipLaunchKernelGGL(ising::k_init_int8, grid, block, 0, (hipStream_t)stream, spins, (uint32_t)L, chunks,
                       n_lanes, (uint32_t)seed, (uint32_t)(seed >> 32));
    return check_launch("k_init_int8");
}

int ising_fill(int8_t* spins, int64_t L, int value, void* stream) {
    if (!spins || !valid_L(L) || !aligned16(spins) || (value != 1 && value != -1)) return ISING_EINVAL;
    const uint64_t n16 = (uint64_t)L * (uint64_t)L / 16u;
    const uint32_t word = value == 1 ? 0x01010101u : 0xFFFFFFFFu;
    uint64_t blocks = (n16 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(ising::k_fill_int8, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, spins,
                       n16, word);
    return check_launch("k_fill_int8");
}

// 3-D lattices (L x L x L, L a power of two in [64, 2048]): the hot start is the square lattice's
// with L^2 rows (r = z L + y) of length L.
int ising3_init(int8_t* spins, int64_t L, uint64_t seed, void* stream) {
    if (!spins || L < 64 || L > 2048 || (L & (L - 1)) != 0 || !aligned16(spins)) return ISING_EINVAL;
    const uint32_t chunks = (uint32_t)((L + 127) / 128);
    const uint64_t n_lanes = (uint64_t)chunks * (uint64_t)L * (uint64_t)L;
    const dim3 grid((unsigned)((n_lanes + 255) / 256)), block(256);
    hipLaunchKernelGGL(ising::k_init_int8, grid, block, 0, (hipStream_t)stream, spins, (uint32_t)L, chunks,
                       n_lanes, (uint32_t)seed, (uint32_t)(seed >> 32));
    return check_launch("k_init_int8");
}

int ising3_fill(int8_t* spins, int64_t L, int value, void* stream) {
    if (!spins || L < 64 || L > 2048 || (L & (L - 1)) != 0 || !aligned16(spins) || (value != 1 && value != -1))
        return ISING_EINVAL;
    const uint64_t n16 = (uint64_t)L * (uint64_t)L * (uint64_t)L / 16u;
    const uint32_t word = value == 1 ? 0x01010101u : 0xFFFFFFFFu;
    hipLaunchKernelGGL(ising::k_fill_int8, dim3((unsigned)std::min<uint64_t>((n16 + 255) / 256, 8192)), dim3(256), 0,
                       (hipStream_t)stream, spins, n16, word);
    return check_launch("k_fill_int8");
}

int ising_half_sweep(int8_t* spins, int64_t L, double beta, uint64_t seed, uint64_t t, int q, void* stream) {
    if (!spins || !valid_L(L) || !aligned16(spins) || !valid_beta(beta) || (q != 0 && q != 1) ||
        t >= (uint64_t(1) << 32))
        return ISING_EINVAL;
    return launch_half_sweep(spins, L, make_thresholds(beta), seed, (uint32_t)t, q, nullptr, (hipStream_t)stream);
}

int ising_sweep(int8_t* spins, int64_t L, double beta, int64_t n_sweeps, uint64_t seed, uint64_t sweep_offset,
                int64_t* trace_ME, void* stream) {
    return ising_sweep_fmt(spins, L, beta, 0, n_sweeps, seed, sweep_offset, trace_ME, stream);
}

int ising_sweep_fmt(int8_t* spins, int64_t L, double beta, int fmt, int64_t n_sweeps, uint64_t seed,
                    uint64_t sweep_offset, int64_t* trace_ME, void* stream) {
    if (!spins || !valid_L(L) || !aligned16(spins) || !valid_beta(beta) || n_sweeps < 0 || fmt < 0 || fmt > 2 ||
        sweep_offset > (uint64_t(1) << 32) || (uint64_t)n_sweeps > (uint64_t(1) << 32) - sweep_offset)
        return ISING_EINVAL;
    return sweep_int8(spins, L, make_thresholds(beta, fmt), n_sweeps, seed, sweep_offset, trace_ME,
                      (hipStream_t)stream, nullptr);
}

int ising_sweep_fused(int8_t* spins, int8_t* scratch, int64_t L, double beta, int fmt, int64_t n_sweeps,
                      uint64_t seed, uint64_t sweep_offset, int64_t* trace_ME, void* stream) {
    if (!spins || !scratch || !valid_L(L) || !aligned16(spins) || !aligned16(scratch) || !valid_beta(beta) ||
        n_sweeps < 0 || fmt < 0 || fmt > 2 || sweep_offset > (uint64_t(1) << 32) ||
        (uint64_t)n_sweeps > (uint64_t(1) << 32) - sweep_offset || !disjoint(spins, scratch, (uint64_t)L * (uint64_t)L))
        return ISING_EINVAL;
    return sweep_fused(spins, scratch, L, make_thresholds(beta, fmt), n_sweeps, seed, sweep_offset, trace_ME,
                       (hipStream_t)stream, nullptr);
}

int ising_sweep_fused_static(int8_t* spins, int64_t L, double beta, int fmt, int64_t n_sweeps, uint64_t seed,
                             uint64_t sweep_offset, int64_t* trace_ME, void* stream) {
    if (!spins || !valid_L(L) || (uint64_t)L * (uint64_t)L > ising::kStaticLatticeBytes || !aligned16(spins) ||
        !valid_beta(beta) || n_sweeps < 0 || fmt < 0 || fmt > 2 || sweep_offset > (uint64_t(1) << 32) ||
        (uint64_t)n_sweeps > (uint64_t(1) << 32) - sweep_offset)
        return ISING_EINVAL;
    int8_t* base = nullptr;
    const int rc = static_scratch(&base);
    if (rc) return rc;
    // the lattice buffer, then the spread sets
    int8_t* const lattice = base;
    int64_t* const sets = reinterpret_cast<int64_t*>(base + ising::kStaticLatticeBytes);
    if (!disjoint_ranges(spins, (uint64_t)L * (uint64_t)L, base, ising::kStaticScratchBytes)) return ISING_EINVAL;
    return sweep_fused(spins, lattice, L, make_thresholds(beta, fmt), n_sweeps, seed, sweep_offset, trace_ME,
                       (hipStream_t)stream, sets);
}

int ising_sweep_fused_step(const int8_t* src, int8_t* dst, int64_t L, double beta, int fmt, uint64_t seed,
                           uint64_t t, int64_t* out_ME, void* stream) {
    if (!src || !dst || !valid_L(L) || !aligned16(src) || !aligned16(dst) || !valid_beta(beta) || fmt < 0 ||
        fmt > 2 || t >= (uint64_t(1) << 32) || !disjoint(src, dst, (uint64_t)L * (uint64_t)L))
        return ISING_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (L > kFusedMaxL || L % 64 != 0) {  // a copy, then the two half-sweeps in place on the copy
        const hipError_t e = hipMemcpyAsync(dst, src, (size_t)L * (size_t)L, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_failed(e, "hipMemcpyAsync");
        return ising_sweep_fmt(dst, L, beta, fmt, 1, seed, t, out_ME, stream);
    }
    if (out_ME) {
        const int rc = zero_trace(out_ME, 2, s);
        if (rc) return rc;
    }
    return launch_fused_sweep(src, dst, L, make_thresholds(beta, fmt), seed, (uint32_t)t, out_ME, s);
}

int ising_sweep_fused_pair(const int8_t* src, int8_t* dst, int64_t L, double beta, int fmt, uint64_t seed,
                           uint64_t t, int64_t* out_ME, void* stream) {
    if (!src || !dst || !valid_L(L) || !aligned16(src) || !aligned16(dst) || !valid_beta(beta) || fmt < 0 ||
        fmt > 2 || t + 1 >= (uint64_t(1) << 32) || !disjoint(src, dst, (uint64_t)L * (uint64_t)L))
        return ISING_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (L % 64 != 0) {  // rows that end in a half group: a copy, then two sweeps in place on the copy
        const hipError_t e = hipMemcpyAsync(dst, src, (size_t)L * (size_t)L, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_failed(e, "hipMemcpyAsync");
        return ising_sweep_fmt(dst, L, beta, fmt, 2, seed, t, out_ME, stream);
    }
    if (out_ME) {
        const int rc = zero_trace(out_ME, 4, s);
        if (rc) return rc;
    }
    if (use_bands(L)) return launch_band_pass(src, dst, L, make_thresholds(beta, fmt), seed, (uint32_t)t, out_ME, s);
    return launch_fused_sweep(src, dst, L, make_thresholds(beta, fmt), seed, (uint32_t)t, out_ME, s, 2);
}

int ising_observables(const int8_t* spins, int64_t L, int64_t* out_ME, void* stream) {
    if (!spins || !out_ME || !valid_L(L) || !aligned16(spins)) return ISING_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(ising::k_zero2, dim3(1), dim3(64), 0, s, out_ME);
    int rc = check_launch("k_zero2");
    if (rc) return rc;
    ising::ObsArgs a;
    a.spins = spins;
    a.L = (uint32_t)L;
    a.groups = groups_of(L);
    a.rows = rows_per_lane(L);
    a.n_lanes = a.groups * (uint32_t)(L / a.rows);
    a.out = out_ME;
    hipLaunchKernelGGL(ising::k_observables_int8, dim3((a.n_lanes + 255u) / 256u), dim3(256), 0, s, a);
    return check_launch("k_observables_int8");
}

int ising_pack(const int8_t* spins, int64_t L, uint32_t* planes, void* stream) {
    if (!spins || !planes || !valid_L(L) || !aligned16(spins) || !aligned16(planes)) return ISING_EINVAL;
    const uint32_t groups = groups_of(L);
    const uint64_t n = (uint64_t)groups * (uint64_t)L;  // up to 2^34 lanes at L = 2^20
    hipLaunchKernelGGL(ising::k_pack, dim3(grid_blocks(n)), dim3(256), 0, (hipStream_t)stream, spins,
                       planes, (uint32_t)L, groups, n);
    return check_launch("k_pack");
}

int ising_unpack(const uint32_t* planes, int64_t L, int8_t* spins, void* stream) {
    if (!spins || !planes || !valid_L(L) || !aligned16(spins) || !aligned16(planes)) return ISING_EINVAL;
    const uint32_t groups = groups_of(L);
    const uint64_t n = (uint64_t)groups * (uint64_t)L;
    hipLaunchKernelGGL(ising::k_unpack, dim3(grid_blocks(n)), dim3(256), 0, (hipStream_t)stream, planes,
                       spins, (uint32_t)L, groups, n);
    return check_launch("k_unpack");
}

int64_t ising_packed_words(int64_t L) {
    if (!valid_L(L)) return ISING_EINVAL;
    return 2 * L * (int64_t)groups_of(L);
}

int ising_fill_packed(uint32_t* planes, int64_t L, int value, void* stream) {
    if (!planes || !valid_L(L) || !aligned16(planes) || (value != 1 && value != -1)) return ISING_EINVAL;
    // a set bit is spin -1; both planes are 2 L G words (the bits past a half group stay zero)
    const uint32_t groups = groups_of(L);
    const uint64_t n = 2ull * (uint64_t)L * groups;
    hipLaunchKernelGGL(ising::k_fill_packed, dim3(grid_blocks(n)), dim3(256), 0, (hipStream_t)stream, planes, n,
                       groups, (uint32_t)(L % 64 != 0), value == 1 ? 0u : 0xFFFFFFFFu);
    return check_launch("k_fill_packed");
}

int ising_init_packed(uint32_t* planes, int64_t L, uint64_t seed, void* stream) {
    if (!planes || !valid_L(L) || !aligned16(planes)) return ISING_EINVAL;
    const uint32_t groups = groups_of(L);
    const uint64_t n = (uint64_t)groups * (uint64_t)L;
    hipLaunchKernelGGL(ising::k_init_packed, dim3(grid_blocks(n)), dim3(256), 0, (hipStream_t)stream,
                       planes, (uint32_t)L, groups, n, (uint32_t)seed, (uint32_t)(seed >> 32));
    return check_launch("k_init_packed");
}


int ising_half_sweep_packed(uint32_t* planes, int64_t L, double beta, uint64_t seed, uint64_t t, int q,
                            void* stream) {
    if (!planes || !valid_L(L) || !aligned16(planes) || !valid_beta(beta) || (q != 0 && q != 1) ||
        t >= (uint64_t(1) << 32))
        return ISING_EINVAL;
    return launch_half_sweep_packed(planes, L, make_thresholds(beta), seed, (uint32_t)t, q, nullptr,
                                    (hipStream_t)stream);
}

int ising_sweep_packed(uint32_t* planes, int64_t L, double beta, int64_t n_sweeps, uint64_t seed,
                       uint64_t sweep_offset, int64_t* trace_ME, void* stream) {
    return ising_sweep_packed_fmt(planes, L, beta, 0, n_sweeps, seed, sweep_offset, trace_ME, stream);
}

int ising_sweep_packed_fmt(uint32_t* planes, int64_t L, double beta, int fmt, int64_t n_sweeps, uint64_t seed,
                           uint64_t sweep_offset, int64_t* trace_ME, void* stream) {
    if (!planes || !valid_L(L) || !aligned16(planes) || !valid_beta(beta) || n_sweeps < 0 || fmt < 0 ||
        fmt > 2 || sweep_offset > (uint64_t(1) << 32) ||
        (uint64_t)n_sweeps > (uint64_t(1) << 32) - sweep_offset)
        return ISING_EINVAL;
    const ising::Thresholds th = make_thresholds(beta, fmt);
    hipStream_t s = (hipStream_t)stream;
    SpreadTrace sp;
    if (trace_ME && n_sweeps > 0) {
        const int rc = sp.begin(nullptr, n_sweeps, s);
        if (rc) return rc;
    }
    for (int64_t i = 0; i < n_sweeps; ++i) {
        const uint32_t t = (uint32_t)(sweep_offset + (uint64_t)i);
        int64_t* set = nullptr;
        if (trace_ME) {
            const int rc = sp.next(trace_ME + 2 * i, 2, &set);
            if (rc) return rc;
        }
        int rc = launch_half_sweep_packed(planes, L, th, seed, t, 1, nullptr, s);
        if (rc) return rc;
        rc = launch_half_sweep_packed(planes, L, th, seed, t, 0, set, s);  // (+ M, E)
        if (rc) return rc;
    }
    return sp.fold();
}

int ising_observables_packed(const uint32_t* planes, int64_t L, int64_t* out_ME, void* stream) {
    if (!planes || !out_ME || !valid_L(L) || !aligned16(planes)) return ISING_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(ising::k_zero2, dim3(1), dim3(64), 0, s, out_ME);
    int rc = check_launch("k_zero2");
    if (rc) return rc;
    const uint32_t groups = groups_of(L);
    const uint64_t n = (uint64_t)groups * (uint64_t)L;
    const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 16384);
    hipLaunchKernelGGL(ising::k_observables_packed, dim3((unsigned)blocks), dim3(256), 0, s, planes, (uint32_t)L,
                       groups, n, out_ME);
    return check_launch("k_observables_packed");
}

int ising_set_option(const char* name, int64_t value) {
    if (!name) return ISING_EINVAL;
    const std::string n(name);
    if (n == "rows_per_lane") {
        if (value != 0 && (value < 2 || value > 64 || (value & (value - 1)) != 0)) return ISING_EINVAL;
        g_opt.rows_per_lane = value;
    } else if (n == "xcd_remap") {
        if (value != 0 && value != 1) return ISING_EINVAL;
        g_opt.xcd_remap = value;
    } else if (n == "nt_store") {
        if (value != 0 && value != 1) return ISING_EINVAL;
        g_opt.nt_store = value;
    } else if (n == "batch_threads") {
        if (value != 0 && value != 256 && value != 512 && value != 1024) return ISING_EINVAL;
        g_opt.batch_threads = value;
    } else if (n == "batch_slab_sites") {
        if (value != 0 && value != -1 && (value < 1024 || value > (1 << 18) || (value & (value - 1)) != 0))
            return ISING_EINVAL;
        g_opt.batch_slab_sites = value;
    } else if (n == "batch_depth") {
        if (value != 0 && value != 1 && value != 2 && value != 4) return ISING_EINVAL;
        g_opt.batch_depth = value;
    } else if (n == "batch_lists_per_cu") {
        if (value != 0 && value != 1 && value != 2) return ISING_EINVAL;
        g_opt.batch_lists_per_cu = value;
    } else if (n == "staged") {
        if (value != 0 && value != 1) return ISING_EINVAL;
        g_opt.staged = value;
    } else if (n == "planes3") {
        if (value != 0 && (value < 2 || value > 256 || (value & (value - 1)) != 0)) return ISING_EINVAL;
        g_opt.planes3 = value;
    } else if (n == "fused_alternate") {
        if (value != 0 && value != 1) return ISING_EINVAL;
        g_opt.fused_alternate = value;
    } else if (n == "fused_sweeps") {
        if (value != 1 && value != 2) return ISING_EINVAL;
        g_opt.fused_sweeps = value;
    } else if (n == "fused_pairs") {
        if (value != 0 && value != 1) return ISING_EINVAL;
        g_opt.fused_pairs = value;
    } else if (n == "fused_ties") {
        if (value != 0 && value != 1) return ISING_EINVAL;
        g_opt.fused_ties = value;
    } else if (n == "packed_ties") {
        if (value != 0 && value != 1) return ISING_EINVAL;
        g_opt.packed_ties = value;
    } else if (n == "ties3") {
        if (value != 0 && value != 1) return ISING_EINVAL;
        g_opt.ties3 = value;
    } else if (n == "fused_bands") {
        if (value < 0 || value > 2) return ISING_EINVAL;
        g_opt.fused_bands = value;
    } else if (n == "band_rows") {
        if (value != 0 && (value < 2 || value > 1024 || (value & (value - 1)) != 0)) return ISING_EINVAL;
        g_opt.band_rows = value;
    } else if (n == "fused_rows") {
        if (value != 0 && (value < 2 || value > 256 || (value & 1) != 0)) return ISING_EINVAL;
        g_opt.fused_rows = value;
    } else {
        return ISING_EINVAL;
    }
    return ISING_OK;
}

int ising_get_option(const char* name, int64_t* value) {
    if (!name || !value) return ISING_EINVAL;
    const std::string n(name);
    if (n == "rows_per_lane") *value = g_opt.rows_per_lane;
    else if (n == "xcd_remap") *value = g_opt.xcd_remap;
    else if (n == "nt_store") *value = g_opt.nt_store;
    else if (n == "staged") *value = g_opt.staged;
    else if (n == "batch_threads") *value = g_opt.batch_threads;
    else if (n == "batch_slab_sites") *value = g_opt.batch_slab_sites;
    else if (n == "batch_depth") *value = g_opt.batch_depth;
    else if (n == "batch_lists_per_cu") *value = g_opt.batch_lists_per_cu;
    else if (n == "fused_rows") *value = g_opt.fused_rows;
    else if (n == "fused_bands") *value = g_opt.fused_bands;
    else if (n == "band_rows") *value = g_opt.band_rows;
    else if (n == "fused_alternate") *value = g_opt.fused_alternate;
    else if (n == "fused_sweeps") *value = g_opt.fused_sweeps;
    else if (n == "fused_ties") *value = g_opt.fused_ties;
    else if (n == "fused_pairs") *value = g_opt.fused_pairs;
    else if (n == "packed_ties") *value = g_opt.packed_ties;
    else if (n == "ties3") *value = g_opt.ties3;
    else if (n == "planes3") *value = g_opt.planes3;
    else return ISING_EINVAL;
    return ISING_OK;
}

int64_t ising_batch_workspace_bytes(const ising_replica_t* replicas, int64_t n) {
    if (!replicas || n <= 0 || n > 65535) return ISING_EINVAL;
    for (int64_t i = 0; i < n; ++i)
        if (!valid_batch_L(replicas[i].L)) return ISING_EINVAL;
    return (int64_t)batch_layout(replicas, n).total;
}

int ising_batch_run(const ising_replica_t* replicas, int64_t n, int64_t n_therm, int64_t n_meas, uint64_t sweep_offset,
                    int fmt, int start, void* workspace, int64_t workspace_bytes, int64_t* trace_ME, double* moments,
                    void* stream) {
    const int64_t need = ising_batch_workspace_bytes(replicas, n);
    if (need < 0 || !workspace || workspace_bytes < need || !aligned16(workspace) || n_therm < 0 || n_meas < 0 ||
        fmt < 0 || fmt > 2 || start < 0 || start > 3 || (uint64_t)(n_therm + n_meas) >= (uint64_t(1) << 31) ||
        sweep_offset > (uint64_t(1) << 32) - (uint64_t)(n_therm + n_meas))
        return ISING_EINVAL;
    for (int64_t i = 0; i < n; ++i)
        if (!valid_beta(replicas[i].beta)) return ISING_EINVAL;
    std::lock_guard<std::mutex> lock(g_batch_mu);
    const BatchLayout lay = batch_layout(replicas, n);
    // replica table (host) -> workspace head (device)
    std::vector<ising::BatchReplica> table((size_t)n);
    uint64_t off = 0;
    for (int64_t i = 0; i < n; ++i) {
        ising::BatchReplica& b = table[(size_t)i];
        std::memset(&b, 0, sizeof b);
        b.L = (uint32_t)replicas[i].L;
        b.W = batch_W(replicas[i].L);
        b.key0 = (uint32_t)replicas[i].seed;
        b.key1 = (uint32_t)(replicas[i].seed >> 32);
        b.t0 = (uint32_t)sweep_offset;
        b.ordered = replicas[i].beta > 0.44068679350977147 ? 1u : 0u;  // ln(1 + sqrt 2) / 2
        b.th = make_thresholds(replicas[i].beta, fmt);
        b.state_off = off;
        off += batch_words(replicas[i].L);
    }
    hipStream_t s = (hipStream_t)stream;
    char* ws = reinterpret_cast<char*>(workspace);
    BatchBuffers bufs{};
    bufs.run = reinterpret_cast<ising::BatchRun*>(ws + lay.params);
    bufs.table = reinterpret_cast<const ising::BatchReplica*>(ws);
    bufs.groups = reinterpret_cast<ising::BatchGroup*>(ws + lay.groups);
    bufs.units = reinterpret_cast<ising::BatchUnit*>(ws + lay.units);
    bufs.state = reinterpret_cast<uint32_t*>(ws + lay.state);
    bufs.exchange = reinterpret_cast<uint64_t*>(ws + lay.exchange);
    bufs.exchange_words = (int64_t)((lay.total - lay.exchange) / 8u);
    hipError_t e = hipMemcpyAsync(ws, table.data(), table.size() * sizeof(ising::BatchReplica),
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_failed(e, "hipMemcpyAsync(replica table)");
    const int cus = compute_units();
    BatchSchedule sched{(int)g_opt.batch_threads, g_opt.batch_slab_sites, (int)g_opt.batch_depth,
                        (int)g_opt.batch_lists_per_cu};
    if (sched.threads == 0 || sched.target == 0 || sched.depth == 0 || sched.per_cu == 0) {
        auto it = g_batch_tuned.find(batch_signature(replicas, n));
        if (it != g_batch_tuned.end()) {
            if (sched.threads == 0) sched.threads = it->second.threads;
            if (sched.target == 0) sched.target = it->second.target;
            if (sched.depth == 0) sched.depth = it->second.depth;
            if (sched.per_cu == 0) sched.per_cu = it->second.per_cu;
        } else if (start == 2) {
            // tuning would overwrite the state being continued
            if (sched.threads == 0) sched.threads = 1024;
            if (sched.target == 0) sched.target = -1;
            if (sched.depth == 0) sched.depth = 1;
            if (sched.per_cu == 0) sched.per_cu = 1;
        } else {
            BatchSchedule tuned{};
            const int rc = autotune_batch(replicas, n, bufs, (uint32_t)start, s, sched, cus, &tuned);
            if (rc) return rc;
            sched = tuned;
        }
    }
    BatchPlan plan = plan_batch(replicas, n, sched.target, (uint32_t)sched.depth, sched.per_cu, cus);
    if (!plan_fits(plan, sched.threads, cus)) plan = plan_batch(replicas, n, -1, 1u, 1, cus);  // unsplit fallback
    if (!plan.ok) return ISING_EINVAL;
    int rc = upload_plan(bufs, plan, s);
    if (rc) return rc;
    rc = set_batch_run(bufs, (uint32_t)start, (uint32_t)n_therm, (uint32_t)n_meas, trace_ME, moments, s);
    if (rc) return rc;
    // One persistent launch (after the clearing of the exchange area), captured once per plan into a
    // hipGraph and replayed on the caller's stream.  The graph holds only what the plan fixes (the
    // workspace's layout, the launch shape); the per-call values come from the workspace.
    char keybuf[320];
    std::snprintf(keybuf, sizeof keybuf, "%p|%zu|%zu|%zu|%zu|%zu|%lld|%d|%zu|%u|%zu", workspace, lay.params, lay.state,
                  lay.groups, lay.units, lay.exchange, (long long)bufs.exchange_words, sched.threads,
                  plan.groups.size(), plan.depth, plan.lds);
    const std::string key(keybuf);
    auto it = g_batch_execs.find(key);
    if (it == g_batch_execs.end()) {
        if (g_batch_execs.size() >= kMaxBatchExecs) {
            // drop the least recently used exec once its latest launch has completed (a wait on that
            // launch alone, not on the device)
            auto lru = g_batch_execs.begin();
            for (auto j = g_batch_execs.begin(); j != g_batch_execs.end(); ++j)
                if (j->second.used < lru->second.used) lru = j;
            e = hipEventSynchronize(lru->second.done);
            if (e != hipSuccess) return hip_failed(e, "hipEventSynchronize");
            (void)hipGraphExecDestroy(lru->second.exec);
            (void)hipEventDestroy(lru->second.done);
            g_batch_execs.erase(lru);
        }
        if (!g_batch_capture) {
            e = hipStreamCreateWithFlags(&g_batch_capture, hipStreamNonBlocking);
            if (e != hipSuccess) return hip_failed(e, "hipStreamCreateWithFlags");
        }
        BatchExec x;
        e = hipEventCreateWithFlags(&x.done, hipEventDisableTiming);
        if (e != hipSuccess) return hip_failed(e, "hipEventCreateWithFlags");
        hipStream_t cs = g_batch_capture;
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) { (void)hipEventDestroy(x.done); return hip_failed(e, "hipStreamBeginCapture"); }
        const int launch_rc = launch_batch(bufs, plan, sched.threads, cs);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(cs, &graph);
        if (launch_rc || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            (void)hipEventDestroy(x.done);
            return launch_rc ? launch_rc : hip_failed(e, "hipStreamEndCapture");
        }
        e = hipGraphInstantiate(&x.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) { (void)hipEventDestroy(x.done); return hip_failed(e, "hipGraphInstantiate"); }
        it = g_batch_execs.emplace(key, x).first;
    }
    it->second.used = ++g_batch_clock;
    e = hipGraphLaunch(it->second.exec, s);
    if (e != hipSuccess) return hip_failed(e, "hipGraphLaunch");
    e = hipEventRecord(it->second.done, s);
    if (e != hipSuccess) return hip_failed(e, "hipEventRecord");
    return ISING_OK;
}

int ising_batch_schedule(const ising_replica_t* replicas, int64_t n, int64_t out[4]) {
    if (!replicas || n <= 0 || !out) return ISING_EINVAL;
    std::lock_guard<std::mutex> lock(g_batch_mu);
    auto it = g_batch_tuned.find(batch_signature(replicas, n));
    if (it == g_batch_tuned.end()) return ISING_EINVAL;
    out[0] = it->second.threads;
    out[1] = it->second.target;
    out[2] = it->second.depth;
    out[3] = it->second.per_cu;
    return ISING_OK;
}

int ising_batch_unpack(const void* workspace, int64_t n, int64_t j, int8_t* spins, void* stream) {
    if (!workspace || !spins || n <= 0 || j < 0 || j >= n || !aligned16(workspace)) return ISING_EINVAL;
    const auto* dtable = reinterpret_cast<const ising::BatchReplica*>(workspace);
    const auto* state =
        reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(workspace) + batch_state_offset(n));
    hipLaunchKernelGGL(ising::k_batch_unpack, dim3(16), dim3(256), 0, (hipStream_t)stream, dtable, state,
                       (uint32_t)j, spins);
    return check_launch("k_batch_unpack");
}

const char* ising_last_error(void) { return g_last_error.c_str(); }

const char* ising_strerror(int status) {
    switch (status) {
        case ISING_OK: return "ok";
        case ISING_EINVAL: return "invalid argument";
        case ISING_EHIP: return "HIP runtime error";
        case ISING_EUNSUPPORTED: return "unsupported";
        default: return "unknown status";
    }
}

int ising_version(void) { return 100; }

}  // extern "C"
