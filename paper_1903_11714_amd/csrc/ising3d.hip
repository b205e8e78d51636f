// ising3d.hip — checkerboard Metropolis sweep of the 3-D Ising model on gfx950.
//
// Paper: Yang, Chen, Roumpos, Colby, Anderson, "High Performance Monte Carlo Simulation of
// Ising Model on TPU Clusters" (arXiv 1903.11714).  Sec. 3 states the Hamiltonian on a
// d-dimensional hypercubic lattice; the checkerboard colouring of Fig. 1 extends to any
// dimension, and the conclusion names the three-dimensional model as the next workload.  Here:
// an L x L x L torus of int8 spins stored z-major (site (z, y, x) at (z L + y) L + x), colour
// q = (x + y + z) mod 2, white (q = 1) then black each sweep, six neighbours, thresholds
// T_s = ceil(2^32 exp(-2 beta s)) for s = 2, 4, 6.  The random numbers are the square lattice's
// with the row index r = z L + y: counter (group, z L + y, sweep, 2m + q).
//
// One colour per launch, in place.  A workgroup owns Y whole rows (y0 .. y0 + Y - 1) of a plane,
// W * 4 KiB contiguous, so every wave moves its rows with the coalesced LDS-regrouped I/O of the
// square-lattice kernels, and walks Rz consecutive planes in z with a three-plane window of bit
// words.  Per plane: the y neighbours are the rows of other lanes (one LDS exchange and one
// workgroup barrier per plane), or, for the workgroup's first and last row when Y < L, rows loaded
// from the neighbouring strip; the x neighbour across a group edge is a bit of the adjacent
// lane's word.  The six-neighbour count is two bit-sliced full adders; the acceptance is the
// bit-plane compare with three thresholds.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "host.hpp"
#include "ising.h"
#include "philox.hpp"
#include "rows.hpp"

namespace ising {

// Thresholds for s = 2, 4, 6 (index 0, 1, 2): low 32 bits, and 1 where T_s = 2^32.
struct Thresholds3 {
    uint32_t t[3];
    uint32_t full[3];
    uint32_t blocks;  // Philox blocks (4 bit planes each) that can decide
};

// The four bit planes of one Philox block against T_2 / T_4 / T_6: the threshold bit is bit
// 31 - k of T_6, flipped on s2 where T_2 differs from it and on s4 where T_4 does.  OR3: the accepted
// sites of each two planes enter acc through one three-input v_bitop3 (as compare_planes<true>; the
// packed sweep, bound by issue, takes it).
template <bool OR3 = false>
__device__ __forceinline__ void compare_planes3(uint32_t& acc, uint32_t& tied, uint32_t s2, uint32_t s4,
                                                const Words4& blk, const Thresholds3& th, uint32_t m) {
    const uint32_t planes[4] = {blk.w0, blk.w1, blk.w2, blk.w3};
    uint32_t won[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const uint32_t k = 4u * m + (uint32_t)w;
        const uint32_t m6 = 0u - ((th.t[2] >> (31u - k)) & 1u);
        const uint32_t d2 = 0u - (((th.t[0] ^ th.t[2]) >> (31u - k)) & 1u);
        const uint32_t d4 = 0u - (((th.t[1] ^ th.t[2]) >> (31u - k)) & 1u);
        // diff = x ^ threshold bit, one uniform mask per instruction (a vector instruction reads at most
        // one scalar register): five instructions per plane
        const uint32_t x = planes[w];
        const uint32_t diff = __builtin_amdgcn_bitop3_b32(__builtin_amdgcn_bitop3_b32(x ^ m6, s2, d2, 0x78), s4, d4, 0x78);
        won[w] = __builtin_amdgcn_bitop3_b32(tied, diff, x, 0x40);  // differs with x = 0: threshold bit 1, x < T
        if (!OR3) acc |= won[w];
        tied = __builtin_amdgcn_bitop3_b32(tied, diff, 0u, 0x30);  // a & ~b
    }
    if (OR3) {
        acc = __builtin_amdgcn_bitop3_b32(acc, won[0], won[1], 0xFE);  // a | b | c
        acc = __builtin_amdgcn_bitop3_b32(acc, won[2], won[3], 0xFE);
    }
}

// ---- Tie queue with three thresholds (as the square lattice's in rows.hpp): entry j = the word's
// tied sites, those of them compared with T_2 and with T_4 (the rest with T_6), its Philox row, and
// update | lane << 2 | group << 8; res[lane] = the sites of the lane's updates 0 .. 3 that the queue
// accepted (zeroed before the pushes).  6 KiB per wave.
struct TieQueue3 {
    uint32_t* task;  // [5][256]
    uint4* res;      // [64]
};
constexpr uint32_t kTieQueue3Bytes = 5u * 256u * 4u + 64u * 16u;

// Anti-aligned neighbours of each site of a word, bit-sliced: c = b0 + 2 b1 + 4 b2 (0 .. 6), from
// two full adders of three neighbours each and their sum.
struct Count3 {
    uint32_t b0, b1, b2;
};

__device__ __forceinline__ Count3 neighbour_count3(uint32_t a, const uint32_t (&nb)[6]) {
    uint32_t x[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) x[k] = a ^ nb[k];
    const uint32_t sa = x[0] ^ x[1] ^ x[2], ca = (x[0] & x[1]) | (x[2] & (x[0] ^ x[1]));
    const uint32_t sb = x[3] ^ x[4] ^ x[5], cb = (x[3] & x[4]) | (x[5] & (x[3] ^ x[4]));
    const uint32_t kk = sa & sb;
    return Count3{sa ^ sb, ca ^ cb ^ kk, (ca & cb) | (kk & (ca ^ cb))};
}

// The start of decide3 for one word whose neighbour count is c: returns the sites decided by the
// count and the first two Philox blocks (to flip at once); tied, s2, s4 = the sites still tied and
// which of them compare with T_2 / T_4.
template <bool OR3 = false>
__device__ __forceinline__ uint32_t decide3_head(const Count3& c, const Thresholds3& th, uint32_t g, uint32_t r,
                                                 uint32_t t, uint32_t q, uint32_t key0, uint32_t key1,
                                                 uint32_t& tied, uint32_t& s2, uint32_t& s4) {
    const uint32_t b0 = c.b0, b1 = c.b1, b2 = c.b2;
    uint32_t sel2 = b1 & ~b0 & ~b2, sel4 = b0 & ~b1 & ~b2, sel6 = ~(b0 | b1 | b2);
    uint32_t acc = b2 | (b1 & b0);  // c >= 3: s <= 0
    if (th.full[0]) { acc |= sel2; sel2 = 0u; }
    if (th.full[1]) { acc |= sel4; sel4 = 0u; }
    if (th.full[2]) { acc |= sel6; sel6 = 0u; }
    tied = sel2 | sel4 | sel6;
#pragma unroll
    for (uint32_t m = 0; m < 2; ++m) {
        if (!wave_any(tied != 0u)) break;
        compare_planes3<OR3>(acc, tied, sel2, sel4, philox4x32_10(g, r, t, 2u * m + q, key0, key1), th, m);
    }
    s2 = sel2;
    s4 = sel4;
    return acc;
}

__device__ __forceinline__ void tq3_push(const TieQueue3& q, uint32_t& n, uint32_t tied, uint32_t s2, uint32_t s4,
                                         uint32_t row, uint32_t meta) {
    const uint64_t B = __builtin_amdgcn_ballot_w64(tied != 0u);
    if (tied != 0u) {
        const uint32_t pos =
            n + __builtin_amdgcn_mbcnt_hi((uint32_t)(B >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)B, 0u));
        q.task[pos] = tied;
        q.task[256u + pos] = s2 & tied;
        q.task[512u + pos] = s4 & tied;
        q.task[768u + pos] = row;
        q.task[1024u + pos] = meta;
    }
    n += (uint32_t)__builtin_popcountll(B);
}

// Settles the n (<= 256) queued words of sweep t, one per lane, from block 2 onwards: all of colour
// QC, or (QC < 0) update u of colour 1 - u % 2 (white first, as in the fused pass).
template <int QC>
__device__ __forceinline__ void tq3_settle(const TieQueue3& q, uint32_t n, const Thresholds3& th, uint32_t t,
                                           uint32_t key0, uint32_t key1, uint32_t lane) {
    wave_lds_sync();
#pragma unroll 1
    for (uint32_t b = 0; b < n; b += 64u) {
        const uint32_t j = b + lane;
        const bool have = j < n;
        uint32_t tied = 0u, t2 = 0u, t4 = 0u, r = 0u, meta = 0u;
        if (have) {
            tied = q.task[j];
            t2 = q.task[256u + j];
            t4 = q.task[512u + j];
            r = q.task[768u + j];
            meta = q.task[1024u + j];
        }
        const uint32_t qc = QC < 0 ? (meta & 1u) ^ 1u : (uint32_t)QC;
        uint32_t acc = 0u;
#pragma unroll 1
        for (uint32_t m = 2; m < th.blocks; ++m) {
            if (!wave_any(tied != 0u)) break;
            compare_planes3(acc, tied, t2, t4, philox4x32_10(meta >> 8, r, t, 2u * m + qc, key0, key1), th, m);
        }
        if (have) reinterpret_cast<uint32_t*>(q.res)[4u * ((meta >> 2) & 63u) + (meta & 3u)] = acc;
    }
    wave_lds_sync();
}

// Exact x < T_s for the sites of sel2 / sel4 / sel6, bit plane by bit plane (as accept_mask).
__device__ __forceinline__ uint32_t accept_mask3(uint32_t sel2, uint32_t sel4, uint32_t sel6, const Thresholds3& th,
                                                 uint32_t g, uint32_t r, uint32_t t, uint32_t q, uint32_t key0,
                                                 uint32_t key1) {
    uint32_t acc = 0;
    if (th.full[0]) { acc |= sel2; sel2 = 0; }
    if (th.full[1]) { acc |= sel4; sel4 = 0; }
    if (th.full[2]) { acc |= sel6; sel6 = 0; }
    uint32_t tied = sel2 | sel4 | sel6;
#pragma unroll 1
    for (uint32_t m = 0; m < th.blocks; ++m) {
        if (!wave_any(tied != 0)) break;
        compare_planes3(acc, tied, sel2, sel4, philox4x32_10(g, r, t, 2u * m + q, key0, key1), th, m);
    }
    return acc;
}

// Metropolis decision for 32 sites a (bit words, site order) with neighbour words nb[0..5].
// c = number of anti-aligned neighbours (0..6), s = 6 - 2c: c >= 3 always flips, c = 2, 1, 0
// compare with T_2, T_4, T_6.  With OBS: anti-aligned bonds of these sites after the update and
// -1 spins among them and `others` (the other colour of the same row segment).
template <bool OBS>
__device__ __forceinline__ uint32_t decide3(uint32_t a, const uint32_t (&nb)[6], uint32_t others, const Thresholds3& th,
                                            uint32_t g, uint32_t r, uint32_t t, uint32_t q, uint32_t key0,
                                            uint32_t key1, Counts& cnt) {
    uint32_t x[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) x[k] = a ^ nb[k];
    const uint32_t s1 = x[0] ^ x[1] ^ x[2], c1 = (x[0] & x[1]) | (x[2] & (x[0] ^ x[1]));
    const uint32_t s2 = x[3] ^ x[4] ^ x[5], c2 = (x[3] & x[4]) | (x[5] & (x[3] ^ x[4]));
    const uint32_t b0 = s1 ^ s2, k0 = s1 & s2;
    const uint32_t b1 = c1 ^ c2 ^ k0, b2 = (c1 & c2) | (k0 & (c1 ^ c2));  // c = b0 + 2 b1 + 4 b2
    const uint32_t ge3 = b2 | (b1 & b0);
    const uint32_t sel2 = b1 & ~b0 & ~b2;
    const uint32_t sel4 = b0 & ~b1 & ~b2;
    const uint32_t sel6 = ~(b0 | b1 | b2);
    const uint32_t F = ge3 | accept_mask3(sel2, sel4, sel6, th, g, r, t, q, key0, key1);
    if (OBS) {
#pragma unroll
        for (int k = 0; k < 6; ++k) cnt.anti += __builtin_popcount(x[k] ^ F);
        cnt.neg += __builtin_popcount(a ^ F) + __builtin_popcount(others);
    }
    return F;
}

struct Sweep3Args {
    int8_t* spins;
    uint32_t L, G;        // G = L / 64 groups per row
    uint32_t Y, ystrips;  // rows per workgroup (W * 4096 / L) and L / Y
    uint32_t Rz;          // planes per workgroup (even, divides L)
    uint32_t t, key0, key1;
    Thresholds3 th;
    int64_t* obs;        // OBS: (M, E) accumulator, zeroed beforehand
    int64_t* zero_slot;  // if non-null, the first workgroup zeroes these two int64
    uint32_t xcd_remap;
};

// HALO: Y < L, so the first and last row of the workgroup take their outer y neighbour from the
// adjacent strip's row in memory; otherwise the workgroup holds whole planes and y wraps inside.
// TQ: the two planes of a loop iteration are updated together -- one exchange and one barrier for
// both, and the words left with tied sites after two Philox blocks settled by the wave at once
// (the planes' colour-Q sites are independent: their z neighbours in each other are the other
// colour).  Same uniforms and results either way.
template <int Q, bool OBS, bool HALO, bool TQ>
__global__ __launch_bounds__(512) void k_sweep3(Sweep3Args a) {
    extern __shared__ uint4 s3_lds[];
    const uint32_t tid = threadIdx.x, nt = blockDim.x, lane = tid & 63u;
    // per wave: row staging (4 KiB), with TQ shared with the tie queue (6 KiB)
    constexpr uint32_t kWave = TQ ? kTieQueue3Bytes / 16u : 256u;
    uint4* const stage = s3_lds + (tid >> 6) * kWave;
    uint2* const xch = reinterpret_cast<uint2*>(s3_lds + (nt >> 6) * kWave);  // two slots of nt words
    uint4* const xch4 = s3_lds + (nt >> 6) * kWave;                           // TQ: two slots of nt entries
    const TieQueue3 q{reinterpret_cast<uint32_t*>(stage), stage + 5u * 64u};
    const uint32_t b = logical_block(blockIdx.x, gridDim.x, a.xcd_remap);
    const uint32_t L = a.L, G = a.G, Y = a.Y, Rz = a.Rz;
    const uint32_t y0 = (b % a.ystrips) * Y, z0 = (b / a.ystrips) * Rz;
    const uint32_t yy = tid / G, g = tid % G, y = y0 + yy;
    if (a.zero_slot && blockIdx.x == 0 && tid == 0) { a.zero_slot[0] = 0; a.zero_slot[1] = 0; }
    const size_t plane = (size_t)L * L;
    const size_t seg = (size_t)y0 * L + (size_t)(tid >> 6) * 4096u;  // this wave's rows in a plane
    // plane of walk step k = 0 .. Rz + 1 (z0 - 1 .. z0 + Rz, wrapped); prefetches past the last
    // one are clamped to it, so every load stays unconditional
    auto zplane = [&](uint32_t k) {
        const uint32_t v = z0 + L - 1 + (k < Rz + 1 ? k : Rz + 1);  // < 2L + 1
        return v >= 2 * L ? v - 2 * L : v >= L ? v - L : v;
    };
    // the outer y neighbour row this lane loads when HALO (lanes in the upper half of the
    // workgroup's rows the row above it, the others the row below)
    const uint32_t hrow = yy < Y / 2 ? (y0 == 0 ? L - 1 : y0 - 1) : (y0 + Y == L ? 0 : y0 + Y);
    auto hplane = [&](uint32_t j) { return z0 + (j < Rz ? j : Rz - 1); };  // plane of halo step j
    auto fetch = [&](Row& raw, uint32_t z) { load_row_coalesced(raw, a.spins + z * plane + seg, lane); };
    auto own = [&](const Row& raw) {
        Row row;
        regroup_to_owner(row, raw, stage, lane);
        return row_bits(row);
    };
    auto fetch_halo = [&](Row& raw, uint32_t z) {
        load_row(raw, a.spins + ((size_t)z * L + hrow) * L + (size_t)g * 64u);
    };
    auto put = [&](uint32_t z, const RowBits& bits) {
        Row row;
        bits_to_row(row, bits);
        store_row_coalesced(a.spins + z * plane + seg, row, stage, lane, false);
    };
    Counts cnt{0u, 0u};
    const uint32_t ir = g + 1 < G ? tid + 1 : tid + 1 - G;  // same row, next group (wrapping)
    const uint32_t il = g > 0 ? tid - 1 : tid + G - 1;      // same row, previous group
    const uint32_t iym = yy > 0 ? tid - G : tid + (Y - 1) * G;
    const uint32_t iyp = yy + 1 < Y ? tid + G : tid - (Y - 1) * G;
    // one plane: prev / cur / next = planes z - 1, z, z + 1 of this lane's row segment, hb = its
    // halo row's bits in plane z
    auto step = [&](uint32_t z, const RowBits& prev, RowBits& cur, const RowBits& next, const RowBits& hb,
                    uint32_t slot) {
        uint2* const x = xch + slot * nt;
        x[tid] = make_uint2(cur.e, cur.o);
        workgroup_lds_sync();
        uint2 ym = x[iym], yp = x[iyp];
        if (HALO && yy == 0) ym = make_uint2(hb.e, hb.o);
        if (HALO && yy + 1 == Y) yp = make_uint2(hb.e, hb.o);
        const uint32_t right_e = x[ir].x, left_o = x[il].y;
        const bool O = ((Q + y + z) & 1u) != 0;  // column parity of this row's colour-Q sites
        const uint32_t sites = O ? cur.o : cur.e, side = O ? cur.e : cur.o;
        const uint32_t hs = O ? shift_next(cur.e, right_e & 1u) : shift_prev(cur.o, left_o >> 31);
        const uint32_t nb[6] = {O ? ym.y : ym.x, O ? yp.y : yp.x, O ? prev.o : prev.e, O ? next.o : next.e,
                                side, hs};
        const uint32_t F = decide3<OBS>(sites, nb, side, a.th, g, z * L + y, a.t, (uint32_t)Q, a.key0, a.key1, cnt);
        if (O) cur.o ^= F; else cur.e ^= F;
        put(z, cur);
    };
    // TQ: planes za and zb = za + 1 (walk order; prev = za - 1, next = zb + 1) in one exchange
    auto step2 = [&](uint32_t za, uint32_t zb, const RowBits& prev, RowBits& ca, RowBits& cb, const RowBits& next,
                     const RowBits& hba, const RowBits& hbb, uint32_t slot) {
        uint4* const x = xch4 + slot * nt;
        x[tid] = make_uint4(ca.e, ca.o, cb.e, cb.o);
        workgroup_lds_sync();
        uint4 ym = x[iym], yp = x[iyp];
        if (HALO && yy == 0) ym = make_uint4(hba.e, hba.o, hbb.e, hbb.o);
        if (HALO && yy + 1 == Y) yp = make_uint4(hba.e, hba.o, hbb.e, hbb.o);
        const uint4 xr = x[ir], xl = x[il];
        const bool Oa = ((Q + y + za) & 1u) != 0, Ob = !Oa;  // L is even, so zb has the other parity
        const uint32_t sa = Oa ? ca.e : ca.o, sb = Ob ? cb.e : cb.o;   // the other colour of each row
        const uint32_t ha = Oa ? shift_next(ca.e, xr.x & 1u) : shift_prev(ca.o, xl.y >> 31);
        const uint32_t hb = Ob ? shift_next(cb.e, xr.z & 1u) : shift_prev(cb.o, xl.w >> 31);
        const uint32_t nba[6] = {Oa ? ym.y : ym.x, Oa ? yp.y : yp.x, Oa ? prev.o : prev.e, Oa ? cb.o : cb.e, sa, ha};
        const uint32_t nbb[6] = {Ob ? ym.w : ym.z, Ob ? yp.w : yp.z, Ob ? ca.o : ca.e, Ob ? next.o : next.e, sb, hb};
        q.res[lane] = make_uint4(0u, 0u, 0u, 0u);
        uint32_t n = 0u, tied, s2, s4;
        uint32_t acc = decide3_head(neighbour_count3(Oa ? ca.o : ca.e, nba), a.th, g, za * L + y, a.t, (uint32_t)Q,
                                    a.key0, a.key1, tied, s2, s4);
        ca.o ^= Oa ? acc : 0u;  // both fields, with selects: the parity is a runtime value
        ca.e ^= Oa ? 0u : acc;
        tq3_push(q, n, tied, s2, s4, za * L + y, 0u | (lane << 2) | (g << 8));
        acc = decide3_head(neighbour_count3(Ob ? cb.o : cb.e, nbb), a.th, g, zb * L + y, a.t, (uint32_t)Q, a.key0,
                           a.key1, tied, s2, s4);
        cb.o ^= Ob ? acc : 0u;
        cb.e ^= Ob ? 0u : acc;
        tq3_push(q, n, tied, s2, s4, zb * L + y, 1u | (lane << 2) | (g << 8));
        tq3_settle<Q>(q, n, a.th, a.t, a.key0, a.key1, lane);
        const uint4 r = q.res[lane];
        ca.o ^= Oa ? r.x : 0u;
        ca.e ^= Oa ? 0u : r.x;
        cb.o ^= Ob ? r.y : 0u;
        cb.e ^= Ob ? 0u : r.y;
        if (OBS) {
            const uint32_t ma = Oa ? ~0u : 0u;  // masks, not selects of fields
            const uint32_t fa = (ca.o & ma) | (ca.e & ~ma), fb = (cb.o & ~ma) | (cb.e & ma);
#pragma unroll
            for (int k = 0; k < 6; ++k) cnt.anti += __builtin_popcount(fa ^ nba[k]) + __builtin_popcount(fb ^ nbb[k]);
            cnt.neg += __builtin_popcount(fa) + __builtin_popcount(sa) + __builtin_popcount(fb) + __builtin_popcount(sb);
        }
        put(za, ca);
        put(zb, cb);
    };
    // prologue: planes z0 - 1 .. z0 + 2 in bits, z0 + 3, z0 + 4 in flight; halo rows of planes
    // z0, z0 + 1 in bits, z0 + 2, z0 + 3 in flight
    Row ra, rb, ha, hb;
    fetch(ra, zplane(0));
    fetch(rb, zplane(1));
    RowBits p = own(ra), c = own(rb);
    fetch(ra, zplane(2));
    fetch(rb, zplane(3));
    RowBits n0 = own(ra), n1 = own(rb);
    fetch(ra, zplane(4));
    fetch(rb, zplane(5));
    RowBits h0{0u, 0u}, h1{0u, 0u};
    if (HALO) {
        fetch_halo(ha, hplane(0));
        fetch_halo(hb, hplane(1));
        h0 = row_bits(ha);
        h1 = row_bits(hb);
        fetch_halo(ha, hplane(2));
        fetch_halo(hb, hplane(3));
    }
#pragma unroll 1
    for (uint32_t k = 0; k < Rz; k += 2) {
        const uint32_t z = zplane(k + 1);
        if (TQ) {
            step2(z, zplane(k + 2), p, c, n0, n1, h0, h1, (k >> 1) & 1u);
            p = n0;
            c = n1;
        } else {
            step(z, p, c, n0, h0, 0);
            p = c;
            c = n0;
            step(zplane(k + 2), p, c, n1, h1, 1);
            p = c;
            c = n1;
        }
        n0 = own(ra);  // planes of walk steps k + 4, k + 5
        n1 = own(rb);
        fetch(ra, zplane(k + 6));
        fetch(rb, zplane(k + 7));
        if (HALO) {
            h0 = row_bits(ha);  // halo rows of planes z + 2, z + 3
            h1 = row_bits(hb);
            fetch_halo(ha, hplane(k + 4));
            fetch_halo(hb, hplane(k + 5));
        }
    }
    if (OBS) block_accumulate(a.obs, cnt.anti, cnt.neg, 1u, 64u * Rz, 3u);
}

// ---- Fused 3-D sweep: both colours of a sweep in one pass, out of place (src -> dst).
//
// A workgroup owns Y rows of every plane of a run of Rz planes and walks it in z.  At step k it
// updates the white sites of plane z0 - 1 + k and then the black sites of the plane before it,
// whose six neighbours (white sites of planes z - 1, z + 1 and of rows y - 1, y + 1, x - 1, x + 1
// of plane z) are final by then (Sec. 3.1, in three dimensions).  A white update reads only values
// the sweep has not changed, so the workgroup recomputes the white sites it needs outside its own
// rows and planes: the planes just before and after its run (from the walk), and, when Y < L, the
// rows just above and below its own in every plane -- one extra wave holds those two halo rows,
// and each halo lane also reads the row beyond its halo row (its outer y neighbour).  One LDS
// exchange per step gives every row its y and x neighbours: the plane being updated as it was,
// and the plane before it after its white update.
struct Fused3Args {
    const int8_t* src;
    int8_t* dst;
    uint32_t L, G;        // G = L / 64 groups per row
    uint32_t Y, ystrips;  // own rows per workgroup and L / Y
    uint32_t Rz;          // planes per workgroup (even, divides L)
    uint32_t t, key0, key1;
    Thresholds3 th;
    int64_t* obs;         // OBS: (M, E) accumulator, zeroed beforehand
    uint32_t xcd_remap;
};

template <bool OBS, bool HALO>
__global__ __launch_bounds__(576) void k_sweep3_fused(Fused3Args a) {
    extern __shared__ uint4 f3_lds[];
    const uint32_t tid = threadIdx.x, nt = blockDim.x, lane = tid & 63u;
    const uint32_t L = a.L, G = a.G, Y = a.Y, Rz = a.Rz, own_n = Y * G;
    uint4* const stage = f3_lds + (tid >> 6) * 256u;                          // own waves: 4 KiB each
    uint4* const xch = f3_lds + (own_n >> 6) * 256u;                          // two slots of nt entries
    const uint32_t b = logical_block(blockIdx.x, gridDim.x, a.xcd_remap);
    const uint32_t y0 = (b % a.ystrips) * Y, z0 = (b / a.ystrips) * Rz;
    const bool own = tid < own_n;
    const uint32_t hh = own ? 0u : (tid - own_n) / G;   // halo lanes: 0 = row above, 1 = row below
    const bool halo = HALO && !own && hh < 2u;          // lanes past the halo rows only shadow
    const uint32_t g = own ? tid % G : (halo ? (tid - own_n) % G : 0u);
    const uint32_t yy = own ? tid / G : 0u;
    const uint32_t wrapy = L - 1u;  // L is a power of two
    const uint32_t y = own ? y0 + yy : (hh == 0u ? (y0 + L - 1u) & wrapy : (y0 + Y) & wrapy);
    const uint32_t yo = hh == 0u ? (y0 + L - 2u) & wrapy : (y0 + Y + 1u) & wrapy;  // halo lanes' outer row
    const size_t plane = (size_t)L * L;
    const size_t seg = (size_t)y0 * L + (size_t)(tid >> 6) * 4096u;          // own waves' rows in a plane
    // plane of walk index k = 0 .. Rz + 3: z0 - 2 .. z0 + Rz + 1, wrapped; prefetches past the last
    // one are clamped to it
    auto zplane = [&](uint32_t k) { return (z0 + L - 2u + (k < Rz + 3u ? k : Rz + 3u)) & wrapy; };
    auto fetch = [&](Row& raw, uint32_t z) {
        if (own) load_row_coalesced(raw, a.src + z * plane + seg, lane);
        else if (halo) load_row(raw, a.src + ((size_t)z * L + y) * L + (size_t)g * 64u);
    };
    auto bits = [&](const Row& raw) {
        if (!own) return halo ? row_bits(raw) : RowBits{0u, 0u};
        Row row;
        regroup_to_owner(row, raw, stage, lane);
        return row_bits(row);
    };
    auto fetch_outer = [&](Row& raw, uint32_t z) {
        if (halo) load_row(raw, a.src + ((size_t)z * L + yo) * L + (size_t)g * 64u);
    };
    auto put = [&](uint32_t z, const RowBits& rb) {
        Row row;
        bits_to_row(row, rb);
        if (own) store_row_coalesced(a.dst + z * plane + seg, row, stage, lane, false);
    };
    // neighbour entries: same row, next / previous group; rows above / below (own rows wrap when
    // the workgroup holds whole planes; otherwise rows 0 and Y - 1 meet the halo lanes, and the
    // halo lanes meet row 0 / Y - 1 on one side and their outer row on the other)
    const bool shadow = !own && !halo;  // lanes past the halo rows read their own entry
    const uint32_t ir = shadow ? tid : (g + 1 < G ? tid + 1 : tid + 1 - G);
    const uint32_t il = shadow ? tid : (g > 0 ? tid - 1 : tid + G - 1);
    uint32_t iym, iyp;
    if (shadow) {
        iym = iyp = tid;
    } else if (own) {
        iym = yy > 0 ? tid - G : (HALO ? own_n + g : tid + (Y - 1) * G);
        iyp = yy + 1 < Y ? tid + G : (HALO ? own_n + G + g : tid - (Y - 1) * G);
    } else {
        iym = hh == 0u ? tid : (Y - 1) * G + g;   // hh == 0: the outer row stands in (below)
        iyp = hh == 0u ? g : tid;                 // hh == 1: the outer row stands in
    }
    Counts cnt{0u, 0u};
    // One step: white sites of plane zw (window p0), then black sites of plane zw - 1 (p1) when B.
    // Planes: pn = zw + 1, p0 = zw, p1 = zw - 1, p2 = zw - 2; out = the halo lanes' outer row of
    // plane zw (black sites as they were).
    auto step = [&](bool B, uint32_t zw, uint32_t slot, const RowBits& pn, RowBits& p0, RowBits& p1, const RowBits& p2,
                    const RowBits& out) {
        uint4* const x = xch + slot * nt;
        x[tid] = make_uint4(p0.e, p0.o, p1.e, p1.o);
        workgroup_lds_sync();
        const bool O = ((1u + y + zw) & 1u) != 0;  // column parity of the white sites of row y of plane zw,
                                                   // and of the black sites of row y of plane zw - 1
        {   // white sites of plane zw (neighbours: black sites as they were)
            uint4 ym = x[iym], yp = x[iyp];
            if (HALO && !own && hh == 0u) ym = make_uint4(out.e, out.o, 0u, 0u);
            if (HALO && !own && hh == 1u) yp = make_uint4(out.e, out.o, 0u, 0u);
            const uint32_t right_e = x[ir].x, left_o = x[il].y;
            const uint32_t sites = O ? p0.o : p0.e, side = O ? p0.e : p0.o;
            const uint32_t hs = O ? shift_next(p0.e, right_e & 1u) : shift_prev(p0.o, left_o >> 31);
            const uint32_t nb[6] = {O ? ym.y : ym.x, O ? yp.y : yp.x, O ? p1.o : p1.e, O ? pn.o : pn.e, side, hs};
            Counts none{0u, 0u};
            const uint32_t F = decide3<false>(sites, nb, side, a.th, g, zw * L + y, a.t, 1u, a.key0, a.key1, none);
            if (O) p0.o ^= F; else p0.e ^= F;
        }
        if (B && own) {   // black sites of plane zw - 1 (neighbours: white sites after this sweep)
            const uint32_t z = (zw + L - 1u) & wrapy;
            const uint4 ym = x[iym], yp = x[iyp];
            const uint32_t right_e = x[ir].z, left_o = x[il].w;
            const uint32_t sites = O ? p1.o : p1.e, side = O ? p1.e : p1.o;
            const uint32_t hs = O ? shift_next(p1.e, right_e & 1u) : shift_prev(p1.o, left_o >> 31);
            const uint32_t nb[6] = {O ? ym.w : ym.z, O ? yp.w : yp.z, O ? p2.o : p2.e, O ? p0.o : p0.e, side, hs};
            const uint32_t F = decide3<OBS>(sites, nb, side, a.th, g, z * L + y, a.t, 0u, a.key0, a.key1, cnt);
            if (O) p1.o ^= F; else p1.e ^= F;
            put(z, p1);
        }
    };
    // prologue: planes z0 - 2, z0 - 1, z0 in bits, z0 + 1, z0 + 2 in flight; outer rows of planes
    // z0 - 1, z0 in bits, z0 + 1, z0 + 2 in flight
    Row ra, rb, oa, ob;
    fetch(ra, zplane(0));
    fetch(rb, zplane(1));
    RowBits p2{0u, 0u}, p1 = bits(ra), p0 = bits(rb);
    fetch(ra, zplane(2));
    RowBits pn = bits(ra);
    fetch(ra, zplane(3));
    fetch(rb, zplane(4));
    RowBits o0{0u, 0u}, o1{0u, 0u};
    if (HALO) {
        fetch_outer(oa, zplane(1));
        fetch_outer(ob, zplane(2));
        o0 = halo ? row_bits(oa) : RowBits{0u, 0u};
        o1 = halo ? row_bits(ob) : RowBits{0u, 0u};
        fetch_outer(oa, zplane(3));
        fetch_outer(ob, zplane(4));
    }
    // steps 0, 1: white sites of planes z0 - 1 and z0 only (plane z0 - 2, z0 - 1 are not this
    // workgroup's to update)
    step(false, zplane(1), 0u, pn, p0, p1, p2, o0);
    p2 = p1; p1 = p0; p0 = pn; pn = bits(ra);
    step(false, zplane(2), 1u, pn, p0, p1, p2, o1);
    p2 = p1; p1 = p0; p0 = pn; pn = bits(rb);
    fetch(ra, zplane(5));
    fetch(rb, zplane(6));
    if (HALO) {
        o0 = halo ? row_bits(oa) : RowBits{0u, 0u};
        o1 = halo ? row_bits(ob) : RowBits{0u, 0u};
        fetch_outer(oa, zplane(5));
        fetch_outer(ob, zplane(6));
    }
    // steps k = 2 .. Rz + 1: white sites of plane z0 - 1 + k, black sites of plane z0 - 2 + k
#pragma unroll 1
    for (uint32_t k = 2; k < Rz + 2; k += 2) {
        step(true, zplane(k + 1), 0u, pn, p0, p1, p2, o0);
        p2 = p1; p1 = p0; p0 = pn; pn = bits(ra);
        step(true, zplane(k + 2), 1u, pn, p0, p1, p2, o1);
        p2 = p1; p1 = p0; p0 = pn; pn = bits(rb);
        fetch(ra, zplane(k + 5));
        fetch(rb, zplane(k + 6));
        if (HALO) {
            o0 = halo ? row_bits(oa) : RowBits{0u, 0u};
            o1 = halo ? row_bits(ob) : RowBits{0u, 0u};
            fetch_outer(oa, zplane(k + 5));
            fetch_outer(ob, zplane(k + 6));
        }
    }
    if (OBS) block_accumulate(a.obs, own ? cnt.anti : 0u, own ? cnt.neg : 0u, own ? 1u : 0u, 64u * Rz, 3u);
}

// ---- The fused 3-D sweep, four independent plane updates per step.  Step j updates the white
// sites of planes w = z0 - 1 + 2j and w + 1 and the black sites of planes w - 3 and w - 2.  The black
// updates' neighbours are white sites of planes the walk finished in earlier steps; the white updates
// read black sites no step has changed yet; and no update reads what another one of its step writes
// (the two white planes meet only at black sites, the two black planes only at white ones).  So one
// exchange and one settle of the wave's tie queue serve all four (as in the square lattice's
// two-sweep pass).  The exchange carries each row's planes w and w + 1 as they were and w - 3, w - 2
// after their white updates.  Same rows read and written as k_sweep3_fused, same uniforms, same
// result.  When Y < L the lanes after the own rows hold the halo rows y0 - 1, y0 + Y (white updates
// only) and then the rows beyond them, y0 - 2 and y0 + Y + 1, which are only read: the halo lanes take
// those rows' old black sites from the exchange like any other row.  Two rows are prefetched a step
// ahead.  Rz must be even.  DIRECT: every lane loads and stores its own 64 bytes (no regroup through
// LDS), which is faster where a wave's 4 KiB span eight or more rows (L <= 512).
template <bool OBS, bool HALO, bool DIRECT>
__global__ __launch_bounds__(640) void k_sweep3_fusedq(Fused3Args a) {
    extern __shared__ uint4 f3q_lds[];
    const uint32_t tid = threadIdx.x, nt = blockDim.x, lane = tid & 63u;
    const uint32_t L = a.L, G = a.G, Y = a.Y, Rz = a.Rz, own_n = Y * G;
    // per wave: row staging (own waves) shared with the tie queue; then two exchange slots of two
    // arrays of one entry per lane
    uint4* const mine = f3q_lds + (tid >> 6) * (kTieQueue3Bytes / 16u);
    uint4* const stage = mine;
    const TieQueue3 q{reinterpret_cast<uint32_t*>(mine), mine + 5u * 64u};
    uint4* const xch = f3q_lds + (nt >> 6) * (kTieQueue3Bytes / 16u);
    const uint32_t b = logical_block(blockIdx.x, gridDim.x, a.xcd_remap);
    const uint32_t y0 = (b % a.ystrips) * Y, z0 = (b / a.ystrips) * Rz;
    const bool own = tid < own_n;                        // uniform per wave (own_n is a multiple of 64)
    // lanes after the own rows: 0 = row y0 - 1, 1 = row y0 + Y (halo), 2 = row y0 - 2, 3 = row
    // y0 + Y + 1 (outer: read only); lanes past those only shadow
    const uint32_t hh = own ? 0u : (tid - own_n) / G;
    const bool halo = HALO && !own && hh < 2u;
    const bool ld = HALO && !own && hh < 4u;             // halo and outer lanes load their row
    const bool act = own || halo;                        // lanes whose white updates are kept
    const uint32_t g = own ? tid % G : (ld ? (tid - own_n) % G : 0u);
    const uint32_t yy = own ? tid / G : 0u;
    const uint32_t wrapy = L - 1u;  // L is a power of two
    const uint32_t yoff[4] = {L - 1u, Y, L - 2u, Y + 1u};
    const uint32_t y = own ? y0 + yy : (y0 + yoff[ld ? hh : 1u]) & wrapy;
    const size_t plane = (size_t)L * L;
    const size_t seg = (size_t)y0 * L + (size_t)(tid >> 6) * 4096u;
    // plane of walk index k = 0 .. Rz + 3: z0 - 2 .. z0 + Rz + 1, wrapped; later ones are clamped
    auto zplane = [&](uint32_t k) { return (z0 + L - 2u + (k < Rz + 3u ? k : Rz + 3u)) & wrapy; };
    auto fetch = [&](Row& raw, uint32_t z) {
        if (own && !DIRECT) load_row_coalesced(raw, a.src + z * plane + seg, lane);
        else if (own || ld) load_row(raw, a.src + ((size_t)z * L + y) * L + (size_t)g * 64u);
    };
    auto bits = [&](const Row& raw) {
        if (DIRECT || !own) return (own || ld) ? row_bits(raw) : RowBits{0u, 0u};
        Row row;
        regroup_to_owner(row, raw, stage, lane);
        return row_bits(row);
    };
    auto put = [&](uint32_t z, const RowBits& rb) {
        Row row;
        bits_to_row(row, rb);
        if (own && DIRECT) store_row(a.dst + ((size_t)z * L + y) * L + (size_t)g * 64u, row, false);
        else if (own) store_row_coalesced(a.dst + z * plane + seg, row, stage, lane, false);
    };
    // neighbour entries (own rows wrap when the workgroup holds whole planes); outer and shadow
    // lanes read their own entry
    const uint32_t ir = !act ? tid : (g + 1 < G ? tid + 1 : tid + 1 - G);
    const uint32_t il = !act ? tid : (g > 0 ? tid - 1 : tid + G - 1);
    uint32_t iym, iyp;
    if (!act) {
        iym = iyp = tid;
    } else if (own) {
        iym = yy > 0 ? tid - G : (HALO ? own_n + g : tid + (Y - 1) * G);
        iyp = yy + 1 < Y ? tid + G : (HALO ? own_n + G + g : tid - (Y - 1) * G);
    } else {
        iym = hh == 0u ? own_n + 2u * G + g : (Y - 1) * G + g;
        iyp = hh == 0u ? g : own_n + 3u * G + g;
    }
    const uint32_t keep = act ? ~0u : 0u;
    Counts cnt{0u, 0u};
    // One white or black update of the sites of parity P (1 = odd columns) of row word pair c;
    // lo, hi = the planes below and above, u = the update's slot in the queue.
    auto update = [&](bool P, RowBits& c, const RowBits& lo, const RowBits& hi, uint32_t ymw, uint32_t ypw,
                      uint32_t re, uint32_t lo_o, uint32_t z, uint32_t colour, uint32_t u, uint32_t mask,
                      uint32_t& n) {
        const uint32_t side = P ? c.e : c.o;
        const uint32_t hs = P ? shift_next(c.e, re & 1u) : shift_prev(c.o, lo_o >> 31);
        const uint32_t nb[6] = {ymw, ypw, P ? lo.o : lo.e, P ? hi.o : hi.e, side, hs};
        uint32_t tied, s2, s4;
        const uint32_t acc = mask & decide3_head(neighbour_count3(P ? c.o : c.e, nb), a.th, g, z * L + y, a.t,
                                                 colour, a.key0, a.key1, tied, s2, s4);
        c.o ^= P ? acc : 0u;
        c.e ^= P ? 0u : acc;
        tq3_push(q, n, mask & tied, s2, s4, z * L + y, u | (lane << 2) | (g << 8));
    };
    // black-update (M, E) terms of the final sites of parity P of c
    auto count = [&](bool P, const RowBits& c, const RowBits& lo, const RowBits& hi, uint32_t ymw, uint32_t ypw,
                     uint32_t re, uint32_t lo_o) {
        const uint32_t mp = P ? ~0u : 0u;  // masks, not selects of fields
        const uint32_t f = (c.o & mp) | (c.e & ~mp), side = (c.e & mp) | (c.o & ~mp);
        const uint32_t hs = P ? shift_next(c.e, re & 1u) : shift_prev(c.o, lo_o >> 31);
        const uint32_t nb[6] = {ymw, ypw, (lo.o & mp) | (lo.e & ~mp), (hi.o & mp) | (hi.e & ~mp), side, hs};
#pragma unroll
        for (int k = 0; k < 6; ++k) cnt.anti += __builtin_popcount(f ^ nb[k]);
        cnt.neg += __builtin_popcount(f) + __builtin_popcount(side);
    };
    // window: q0 .. q6 = planes w - 4 .. w + 2
    Row ra, rb;
    fetch(ra, zplane(0));
    fetch(rb, zplane(1));
    RowBits q0{0u, 0u}, q1{0u, 0u}, q2{0u, 0u}, q3 = bits(ra), q4 = bits(rb);
    fetch(ra, zplane(2));
    fetch(rb, zplane(3));
    RowBits q5 = bits(ra), q6 = bits(rb);
    fetch(ra, zplane(4));
    fetch(rb, zplane(5));
    const uint32_t steps = Rz / 2u + 2u;
#pragma unroll 1
    for (uint32_t j = 0; j < steps; ++j) {
        const bool WH = j <= Rz / 2u, BL = j >= 2u && own;
        const uint32_t w = zplane(2u * j + 1u);
        uint4* const xw = xch + (j & 1u) * 2u * nt;  // planes w, w + 1 as they were
        uint4* const xb = xw + nt;                      // planes w - 3, w - 2 after their white updates
        xw[tid] = make_uint4(q4.e, q4.o, q5.e, q5.o);
        xb[tid] = make_uint4(q1.e, q1.o, q2.e, q2.o);
        workgroup_lds_sync();
        const bool O = ((1u + y + w) & 1u) != 0;  // column parity of the white sites of row y of plane w
                                                   // and of the black sites of row y of plane w - 3
        q.res[lane] = make_uint4(0u, 0u, 0u, 0u);
        uint32_t n = 0u;
        if (WH) {
            const uint4 ym = xw[iym], yp = xw[iyp], xr = xw[ir], xl = xw[il];
            update(O, q4, q3, q5, O ? ym.y : ym.x, O ? yp.y : yp.x, xr.x, xl.y, w, 1u, 0u, keep, n);
            update(!O, q5, q4, q6, O ? ym.z : ym.w, O ? yp.z : yp.w, xr.z, xl.w, (w + 1u) & wrapy, 1u, 2u, keep, n);
        }
        const uint32_t zb = (w + L - 3u) & wrapy;
        uint4 ym{}, yp{}, xr{}, xl{};
        if (BL) {
            ym = xb[iym];
            yp = xb[iyp];
            xr = xb[ir];
            xl = xb[il];
            update(O, q1, q0, q2, O ? ym.y : ym.x, O ? yp.y : yp.x, xr.x, xl.y, zb, 0u, 1u, ~0u, n);
            update(!O, q2, q1, q3, O ? ym.z : ym.w, O ? yp.z : yp.w, xr.z, xl.w, (zb + 1u) & wrapy, 0u, 3u, ~0u, n);
        }
        tq3_settle<-1>(q, n, a.th, a.t, a.key0, a.key1, lane);
        const uint4 r = q.res[lane];  // zero for an update the step does not make
        q4.o ^= O ? r.x : 0u;
        q4.e ^= O ? 0u : r.x;
        q5.o ^= O ? 0u : r.z;
        q5.e ^= O ? r.z : 0u;
        if (BL) {
            q1.o ^= O ? r.y : 0u;
            q1.e ^= O ? 0u : r.y;
            q2.o ^= O ? 0u : r.w;
            q2.e ^= O ? r.w : 0u;
            if (OBS) {
                count(O, q1, q0, q2, O ? ym.y : ym.x, O ? yp.y : yp.x, xr.x, xl.y);
                count(!O, q2, q1, q3, O ? ym.z : ym.w, O ? yp.z : yp.w, xr.z, xl.w);
            }
            put(zb, q1);
            put((zb + 1u) & wrapy, q2);
        }
        q0 = q2;
        q1 = q3;
        q2 = q4;
        q3 = q5;
        q4 = q6;
        q5 = bits(ra);  // planes of walk index 2j + 4, 2j + 5
        q6 = bits(rb);
        fetch(ra, zplane(2u * j + 6u));
        fetch(rb, zplane(2u * j + 7u));
    }
    if (OBS) block_accumulate(a.obs, own ? cnt.anti : 0u, own ? cnt.neg : 0u, own ? 1u : 0u, 64u * Rz, 3u);
}

// (M, E) of a cubic lattice: each lane one 64-column group of one row; bonds to +x, +y, +z.
__global__ __launch_bounds__(256) void k_observables3(const int8_t* spins, uint32_t L, uint32_t G, uint64_t n_lanes,
                                                      int64_t* out) {
    const uint64_t id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = id < n_lanes;
    uint32_t anti = 0, neg = 0;
    if (active) {
        const uint32_t g = (uint32_t)(id % G);
        const uint64_t r = id / G;  // z L + y
        const uint32_t z = (uint32_t)(r / L), y = (uint32_t)(r % L);
        const uint32_t gr = g + 1 == G ? 0 : g + 1;
        const size_t base = (size_t)r * L;
        const size_t down = ((size_t)z * L + (y + 1 == L ? 0 : y + 1)) * L;
        const size_t back = ((size_t)(z + 1 == L ? 0 : z + 1) * L + y) * L;
        Row cur, dn, bk;
        load_row(cur, spins + base + (size_t)g * 64u);
        load_row(dn, spins + down + (size_t)g * 64u);
        load_row(bk, spins + back + (size_t)g * 64u);
        const uint32_t right = *reinterpret_cast<const uint32_t*>(spins + base + (size_t)gr * 64u);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const uint32_t nbw = k < 15 ? cur.d[k + 1] : right;
            const uint32_t rn = __builtin_amdgcn_alignbyte(nbw, cur.d[k], 1);  // right neighbours
            neg += __builtin_popcount(cur.d[k] & 0x80808080u);
            anti += __builtin_popcount((cur.d[k] ^ rn) & 0x80808080u);
            anti += __builtin_popcount((cur.d[k] ^ dn.d[k]) & 0x80808080u);
            anti += __builtin_popcount((cur.d[k] ^ bk.d[k]) & 0x80808080u);
        }
    }
    block_accumulate(out, anti, neg, active ? 1u : 0u, 64u, 3u);
}

// ---- 1-bit layout in 3-D: the square lattice's packed layout over the L^2 rows r = z L + y.
// Plane q holds, for every row r and group g, the word of the 32 colour-q sites of the group
// (bit p(i) for site i, set = spin -1); word index (q L^2 + r) G + g.  Colour q of row (z, y) sits
// at column parity (q + y + z) mod 2.
__device__ __forceinline__ uint32_t row_parity3(uint32_t r, uint32_t L) { return ((r / L) + r) & 1u; }

__global__ __launch_bounds__(256) void k_pack3(const int8_t* spins, uint32_t* planes, uint32_t L, uint32_t G,
                                               uint64_t n_lanes) {
    const uint64_t id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n_lanes) return;
    const uint32_t g = (uint32_t)(id % G), r = (uint32_t)(id / G);
    Row row;
    load_row(row, spins + (size_t)r * L + (size_t)g * 64u);
    const uint32_t even = site_bits<0>(row), odd = site_bits<1>(row), par = row_parity3(r, L);
    const size_t rows = (size_t)L * L;
    planes[(size_t)r * G + g] = par ? odd : even;           // q = 0 at column parity par
    planes[(rows + r) * G + g] = par ? even : odd;          // q = 1
}

__global__ __launch_bounds__(256) void k_unpack3(const uint32_t* planes, int8_t* spins, uint32_t L, uint32_t G,
                                                 uint64_t n_lanes) {
    const uint64_t id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n_lanes) return;
    const uint32_t g = (uint32_t)(id % G), r = (uint32_t)(id / G);
    const size_t rows = (size_t)L * L;
    const uint32_t q0 = planes[(size_t)r * G + g], q1 = planes[(rows + r) * G + g];
    const uint32_t par = row_parity3(r, L);
    RowBits b;
    b.e = par ? q1 : q0;
    b.o = par ? q0 : q1;
    Row row;
    bits_to_row(row, b);
    store_row(spins + (size_t)r * L + (size_t)g * 64u, row, false);
}

// packed hot start: the int8 hot start's bits of one group (row r = z L + y), split by colour
__global__ __launch_bounds__(256) void k_init_packed3(uint32_t* planes, uint32_t L, uint32_t G, uint64_t n_lanes,
                                                      uint32_t key0, uint32_t key1) {
    const uint64_t id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n_lanes) return;
    const uint32_t g = (uint32_t)(id % G), r = (uint32_t)(id / G);
    const Words4 w = philox4x32_10(g >> 1, r, 0u, 0x80000000u, key0, key1);
    const uint32_t lo = (g & 1u) ? w.w2 : w.w0, hi = (g & 1u) ? w.w3 : w.w1;  // columns 0-31, 32-63
    // bit c of (lo, hi) set = spin -1 at column c; gather the even and the odd columns in site order
    Row row;
#pragma unroll
    for (int d = 0; d < 16; ++d) {
        const uint32_t src = d < 8 ? lo : hi;
        const uint32_t nib = (src >> (4 * (d & 7))) & 15u;
        row.d[d] = ((nib & 1u) ? 0xFFu : 0x01u) | ((nib & 2u) ? 0xFF00u : 0x0100u) |
                   ((nib & 4u) ? 0xFF0000u : 0x010000u) | ((nib & 8u) ? 0xFF000000u : 0x01000000u);
    }
    const uint32_t even = site_bits<0>(row), odd = site_bits<1>(row), par = row_parity3(r, L);
    const size_t rows = (size_t)L * L;
    planes[(size_t)r * G + g] = par ? odd : even;
    planes[(rows + r) * G + g] = par ? even : odd;
}

struct Packed3Args {
    uint32_t* planes;
    uint32_t L, G, Rz;   // Rz planes per lane (even, divides L)
    uint64_t n_lanes;    // L * G * (L / Rz): lane = ((zs * L + y) * G + g)
    uint32_t t, key0, key1;
    Thresholds3 th;
    int64_t* obs;  // OBS: a spread set (zeroed beforehand) that takes (M, E)
    uint32_t xcd_remap;
};

// Half-sweep of colour Q on the packed layout: a lane owns group g of row y and walks Rz planes in
// z.  The six neighbours of its 32 colour-Q sites are the other plane's words of rows (z, y +- 1),
// (z +- 1, y) in the same group, of row (z, y) itself, and that word shifted by one site with the
// edge bit from the adjacent group.  Consecutive lanes take consecutive groups and rows of a plane,
// so every load of a wave is one contiguous run of words.
template <int Q, bool OBS>
__global__ __launch_bounds__(256) void k_sweep3_packed(Packed3Args a) {
    const uint64_t id = (uint64_t)logical_block(blockIdx.x, gridDim.x, a.xcd_remap) * blockDim.x + threadIdx.x;
    const bool active = id < a.n_lanes;
    Counts cnt{0u, 0u};
    if (active) {
        const uint32_t L = a.L, G = a.G, Rz = a.Rz;
        const uint32_t g = (uint32_t)(id % G);
        const uint64_t zy = id / G;
        const uint32_t y = (uint32_t)(zy % L), z0 = (uint32_t)(zy / L) * Rz;
        const uint32_t gl = g == 0 ? G - 1 : g - 1, gr = g + 1 == G ? 0 : g + 1;
        const uint32_t ym = y == 0 ? L - 1 : y - 1, yp = y + 1 == L ? 0 : y + 1;
        const size_t rows = (size_t)L * L;
        uint32_t* const pq = a.planes + (size_t)Q * rows * G;
        const uint32_t* const po = a.planes + (size_t)(1 - Q) * rows * G;
        auto word = [&](const uint32_t* p, uint32_t z, uint32_t yy, uint32_t gg) {
            return p[((size_t)z * L + yy) * G + gg];
        };
        uint32_t zprev = word(po, z0 == 0 ? L - 1 : z0 - 1, y, g);
        uint32_t zcur = word(po, z0, y, g);
#pragma unroll 1
        for (uint32_t k = 0; k < Rz; ++k) {
            const uint32_t z = z0 + k, zn = z + 1 == L ? 0 : z + 1;
            const uint32_t zpn = word(po, zn, y, g);
            const uint32_t sites = word(pq, z, y, g);
            const uint32_t up = word(po, z, ym, g), dn = word(po, z, yp, g);
            const bool O = ((Q + y + z) & 1u) != 0;  // column parity of the colour-Q sites of row (z, y)
            const uint32_t edge = word(po, z, y, O ? gr : gl);
            const uint32_t hs = O ? shift_next(zcur, edge & 1u) : shift_prev(zcur, edge >> 31);
            const uint32_t nb[6] = {up, dn, zprev, zpn, zcur, hs};
            const uint32_t F = decide3<OBS>(sites, nb, zcur, a.th, g, z * L + y, a.t, (uint32_t)Q, a.key0, a.key1, cnt);
            pq[((size_t)z * L + y) * G + g] = sites ^ F;
            zprev = zcur;
            zcur = zpn;
        }
    }
    if (OBS) block_accumulate(spread_line(a.obs, blockIdx.x), cnt.anti, cnt.neg, active ? 1u : 0u, 64u * a.Rz, 3u);
}

// Half-sweep of colour Q on the packed cubic layout with the ties of four planes settled together:
// a lane takes planes z .. z + 3 of its column at a time (all colour-Q sites of a half-sweep are
// independent), draws the first two Philox blocks of each word, queues the words still holding tied
// sites and settles them with the other lanes'.  Same uniforms and results as k_sweep3_packed.
// Rz % 4 == 0; lanes past n_lanes shadow the last lane without storing.  OBS: (M, E) of the lattice
// as the launch finds it, before its own updates, from the neighbour counts the update forms anyway
// (k_sweep3_packed counts after its updates instead).
template <int Q, bool OBS>
__global__ __launch_bounds__(256) void k_sweep3_packed_q(Packed3Args a) {
    extern __shared__ uint4 packed3_lds[];
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    uint4* const mine = packed3_lds + (tid >> 6) * (kTieQueue3Bytes / 16u);
    const TieQueue3 q{reinterpret_cast<uint32_t*>(mine), mine + 5u * 64u};
    const uint64_t raw = (uint64_t)logical_block(blockIdx.x, gridDim.x, a.xcd_remap) * blockDim.x + tid;
    const bool active = raw < a.n_lanes;
    const uint64_t id = active ? raw : a.n_lanes - 1u;
    uint32_t n1 = 0u, n2 = 0u, neg = 0u;  // OBS: anti-aligned bonds = n1 + 2 n2; -1 spins
    const uint32_t L = a.L, G = a.G, Rz = a.Rz;
    const uint32_t g = (uint32_t)(id % G);
    const uint64_t zy = id / G;
    const uint32_t y = (uint32_t)(zy % L), z0 = (uint32_t)(zy / L) * Rz;
    const uint32_t gl = g == 0 ? G - 1 : g - 1, gr = g + 1 == G ? 0 : g + 1;
    const uint32_t ym = y == 0 ? L - 1 : y - 1, yp = y + 1 == L ? 0 : y + 1;
    const size_t rows = (size_t)L * L;
    uint32_t* const pq = a.planes + (size_t)Q * rows * G;
    const uint32_t* const po = a.planes + (size_t)(1 - Q) * rows * G;
    auto at = [&](uint32_t z, uint32_t yy, uint32_t gg) { return ((size_t)z * L + yy) * G + gg; };
    uint32_t zprev = po[at(z0 == 0 ? L - 1 : z0 - 1, y, g)];
    uint32_t zcur = po[at(z0, y, g)];
    const Thresholds3& th = a.th;
#pragma unroll 1
    for (uint32_t k0 = 0; k0 < Rz; k0 += 4) {
        uint32_t zw[6], w[4], up[4], dn[4], ed[4];
        zw[0] = zprev;
        zw[1] = zcur;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t z = z0 + k0 + (uint32_t)i, zn = z + 1 == L ? 0 : z + 1;
            const bool O = ((Q + y + z) & 1u) != 0;  // column parity of the colour-Q sites of row (z, y)
            zw[i + 2] = po[at(zn, y, g)];
            w[i] = pq[at(z, y, g)];
            up[i] = po[at(z, ym, g)];
            dn[i] = po[at(z, yp, g)];
            ed[i] = po[at(z, y, O ? gr : gl)];
        }
        q.res[lane] = make_uint4(0u, 0u, 0u, 0u);
        uint32_t n = 0u;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t z = z0 + k0 + (uint32_t)i;
            const bool O = ((Q + y + z) & 1u) != 0;
            const uint32_t side = zw[i + 1];
            const uint32_t hs = O ? shift_next(side, ed[i] & 1u) : shift_prev(side, ed[i] >> 31);
            const uint32_t nb[6] = {up[i], dn[i], zw[i], zw[i + 2], side, hs};
            const Count3 c = neighbour_count3(w[i], nb);
            if (OBS) {
                // the lattice as the launch finds it: the anti-aligned neighbours of each colour-Q site
                // (every bond once), and the spins of both colours
                n1 += __builtin_popcount(c.b0);
                n2 += __builtin_popcount(c.b1) + 2u * __builtin_popcount(c.b2);
                neg += __builtin_popcount(w[i]) + __builtin_popcount(side);
                // keep the counts here rather than sunk past the Philox blocks with their inputs
                __asm__ volatile("" : "+v"(n1), "+v"(n2), "+v"(neg));
            }
            uint32_t tied, s2, s4;
            w[i] ^= decide3_head<true>(c, th, g, z * L + y, a.t, (uint32_t)Q, a.key0, a.key1, tied, s2, s4);
            tq3_push(q, n, tied, s2, s4, z * L + y, (uint32_t)i | (lane << 2) | (g << 8));
        }
        tq3_settle<Q>(q, n, th, a.t, a.key0, a.key1, lane);
        const uint4 rr = q.res[lane];
        w[0] ^= rr.x;
        w[1] ^= rr.y;
        w[2] ^= rr.z;
        w[3] ^= rr.w;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (active) pq[at(z0 + k0 + (uint32_t)i, y, g)] = w[i];
        }
        zprev = zw[4];
        zcur = zw[5];
    }
    // a lane's counts stay below 2^13 (Rz <= 32 words of 32 sites, six bonds each)
    if (OBS)
        block_accumulate(spread_line(a.obs, blockIdx.x), active ? n1 + 2u * n2 : 0u, active ? neg : 0u,
                         active ? 1u : 0u, 64u * a.Rz, 3u);
}

// (M, E) of a packed cubic lattice: every bond has one black end, so the black sites' anti-aligned
// neighbour counts cover all 3 L^3 bonds once.
__global__ __launch_bounds__(256) void k_observables3_packed(const uint32_t* planes, uint32_t L, uint32_t G,
                                                             uint64_t n_lanes, int64_t* out, uint32_t spread) {
    const uint64_t id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = id < n_lanes;
    uint32_t anti = 0, neg = 0;
    if (active) {
        const uint32_t g = (uint32_t)(id % G);
        const uint32_t r = (uint32_t)(id / G), z = r / L, y = r % L;
        const uint32_t gl = g == 0 ? G - 1 : g - 1, gr = g + 1 == G ? 0 : g + 1;
        const size_t rows = (size_t)L * L;
        const uint32_t* p0 = planes;
        const uint32_t* p1 = planes + rows * G;
        auto w1 = [&](uint32_t zz, uint32_t yy, uint32_t gg) { return p1[((size_t)zz * L + yy) * G + gg]; };
        const uint32_t b = p0[(size_t)r * G + g], w = w1(z, y, g);
        const bool O = ((y + z) & 1u) != 0;  // column parity of the black sites of row (z, y)
        const uint32_t hs = O ? shift_next(w, w1(z, y, gr) & 1u) : shift_prev(w, w1(z, y, gl) >> 31);
        anti = __builtin_popcount(b ^ w) + __builtin_popcount(b ^ hs) +
               __builtin_popcount(b ^ w1(z, y == 0 ? L - 1 : y - 1, g)) +
               __builtin_popcount(b ^ w1(z, y + 1 == L ? 0 : y + 1, g)) +
               __builtin_popcount(b ^ w1(z == 0 ? L - 1 : z - 1, y, g)) +
               __builtin_popcount(b ^ w1(z + 1 == L ? 0 : z + 1, y, g));
        neg = __builtin_popcount(b) + __builtin_popcount(w);
    }
    // spread: out is a spread set (a line per workgroup)
    block_accumulate(spread ? spread_line(out, blockIdx.x) : out, anti, neg, active ? 1u : 0u, 64u, 3u);
}

}  // namespace ising

// ==========================================================================================
// Host side.
namespace {

// 3-D lattices: L a power of two, 64 <= L <= 2048 (a wave's 4 KiB is then whole rows).
bool valid_L3(int64_t L) { return L >= 64 && L <= 2048 && (L & (L - 1)) == 0; }

void host_thresholds3(double beta, uint64_t T[3]) {
    for (int k = 0; k < 3; ++k) {
        const double s = 2.0 * (k + 1);
        double y = std::ceil(std::ldexp(std::exp(-2.0 * beta * s), 32));
        if (y > 4294967296.0) y = 4294967296.0;
        if (!(y >= 0.0)) y = 0.0;
        T[k] = (uint64_t)y;
    }
}

ising::Thresholds3 make_thresholds3(double beta) {
    uint64_t T[3];
    host_thresholds3(beta, T);
    ising::Thresholds3 th;
    for (int k = 0; k < 3; ++k) {
        th.full[k] = T[k] >= (uint64_t(1) << 32);
        th.t[k] = th.full[k] ? 0u : (uint32_t)T[k];
    }
    th.blocks = 8;
    return th;
}

struct Shape3 {
    uint32_t W, Y, ystrips, Rz;
};

// W waves per workgroup (whole planes up to 4 waves, 8 waves from L = 1024), Y = W * 4096 / L
// rows; Rz planes per workgroup: the tallest even divisor of L up to 128 that keeps >= 2048 waves (two
// per SIMD).  Taller walks re-read fewer planes (measured against up to 32 planes and 4096 waves: 512^3
// +9% at 16 planes, 1024^3 +5% at 128, 2048^3 +0.5%; a walk that leaves one wave per SIMD ran slower).
Shape3 shape3(int64_t L) {
    Shape3 s;
    const uint64_t waves_per_plane = (uint64_t)L * (uint64_t)L / 4096u;
    s.W = (uint32_t)std::min<uint64_t>(waves_per_plane, L >= 1024 ? 8u : 4u);
    s.Y = (uint32_t)(s.W * 4096u / (uint64_t)L);
    s.ystrips = (uint32_t)(L / s.Y);
    const int64_t forced = ising_host::option("planes3");
    if (forced > 0 && L % forced == 0) {
        s.Rz = (uint32_t)forced;
        return s;
    }
    uint32_t Rz = 128;
    while (Rz > 2 && (waves_per_plane * (uint64_t)(L / Rz) < 2048u || L % Rz != 0)) Rz >>= 1;
    s.Rz = Rz;
    return s;
}

int launch_half_sweep3(int8_t* spins, int64_t L, const ising::Thresholds3& th, uint64_t seed, uint32_t t, int q,
                       int64_t* obs, int64_t* zero_slot, hipStream_t stream) {
    const Shape3 sh = shape3(L);
    ising::Sweep3Args a;
    a.spins = spins;
    a.L = (uint32_t)L;
    a.G = (uint32_t)(L / 64);
    a.Y = sh.Y;
    a.ystrips = sh.ystrips;
    a.Rz = sh.Rz;
    a.t = t;
    a.key0 = (uint32_t)seed;
    a.key1 = (uint32_t)(seed >> 32);
    a.th = th;
    a.obs = obs;
    a.zero_slot = zero_slot;
    a.xcd_remap = ising_host::xcd_remap() ? 1u : 0u;
    const uint32_t threads = sh.W * 64u;
    const bool tq = ising_host::option("ties3") != 0;
    const size_t lds = tq ? (size_t)sh.W * ising::kTieQueue3Bytes + 2u * threads * sizeof(uint4)
                          : (size_t)sh.W * 4096u + 2u * threads * sizeof(uint2);
    const dim3 grid(sh.ystrips * (uint32_t)(L / sh.Rz)), block(threads);
    const bool halo = (int64_t)sh.Y < L;
#define ISING_LAUNCH3(QQ, OO, HH)                                                                         \
    do {                                                                                                  \
        if (tq) hipLaunchKernelGGL((ising::k_sweep3<QQ, OO, HH, true>), grid, block, lds, stream, a);    \
        else hipLaunchKernelGGL((ising::k_sweep3<QQ, OO, HH, false>), grid, block, lds, stream, a);      \
    } while (0)
    if (q == 1) {
        if (halo) { if (obs) ISING_LAUNCH3(1, true, true); else ISING_LAUNCH3(1, false, true); }
        else { if (obs) ISING_LAUNCH3(1, true, false); else ISING_LAUNCH3(1, false, false); }
    } else {
        if (halo) { if (obs) ISING_LAUNCH3(0, true, true); else ISING_LAUNCH3(0, false, true); }
        else { if (obs) ISING_LAUNCH3(0, true, false); else ISING_LAUNCH3(0, false, false); }
    }
#undef ISING_LAUNCH3
    return ising_host::check_launch("k_sweep3");
}

// planes per lane of the packed 3-D sweep: the tallest even divisor of L up to 16 that leaves
// >= 4096 waves (option "planes3" applies here too; at 1024^3, 16 planes ran 2% faster than 32, 8 and
// 64 slower)
uint32_t packed_planes3(int64_t L) {
    const int64_t forced = ising_host::option("planes3");
    if (forced > 0 && L % forced == 0) return (uint32_t)forced;
    const uint64_t lanes_per_plane = (uint64_t)L * (uint64_t)(L / 64);
    uint32_t Rz = 16;
    while (Rz > 2 && lanes_per_plane * (uint64_t)(L / Rz) < 4096u * 64u) Rz >>= 1;
    return Rz;
}

// The launch shape of a call's packed half-sweeps, read from the options once per call, so that
// every launch of the call takes the same kernel (the two kernels count (M, E) at different points).
struct Packed3Plan {
    uint32_t Rz;
    bool ties;  // k_sweep3_packed_q: counts the lattice as it finds it
};

Packed3Plan packed3_plan(int64_t L) {
    const uint32_t Rz = packed_planes3(L);
    return Packed3Plan{Rz, ising_host::option("packed_ties") != 0 && Rz % 4u == 0};
}

using Packed3Kernel = void (*)(ising::Packed3Args);

Packed3Kernel pick_packed3(bool ties, int q, bool obs) {
    if (ties)
        return q == 1 ? (obs ? ising::k_sweep3_packed_q<1, true> : ising::k_sweep3_packed_q<1, false>)
                      : (obs ? ising::k_sweep3_packed_q<0, true> : ising::k_sweep3_packed_q<0, false>);
    return q == 1 ? (obs ? ising::k_sweep3_packed<1, true> : ising::k_sweep3_packed<1, false>)
                  : (obs ? ising::k_sweep3_packed<0, true> : ising::k_sweep3_packed<0, false>);
}

// obs: null, or a zeroed spread set for (M, E) (after the launch's updates for k_sweep3_packed, before
// them for k_sweep3_packed_q)
int launch_half_sweep3_packed(uint32_t* planes, int64_t L, const Packed3Plan& plan, const ising::Thresholds3& th,
                              uint64_t seed, uint32_t t, int q, int64_t* obs, hipStream_t stream) {
    ising::Packed3Args a;
    a.planes = planes;
    a.L = (uint32_t)L;
    a.G = (uint32_t)(L / 64);
    a.Rz = plan.Rz;
    a.n_lanes = (uint64_t)L * a.G * (uint64_t)(L / a.Rz);
    a.t = t;
    a.key0 = (uint32_t)seed;
    a.key1 = (uint32_t)(seed >> 32);
    a.th = th;
    a.obs = obs;
    a.xcd_remap = ising_host::xcd_remap() ? 1u : 0u;
    const dim3 grid((unsigned)((a.n_lanes + 255) / 256)), block(256);
    const size_t lds = plan.ties ? 4u * ising::kTieQueue3Bytes : 0u;  // four waves per workgroup
    const Packed3Kernel kern = pick_packed3(plan.ties, q, obs != nullptr);
    void* args[] = {&a};
    const hipError_t e = hipLaunchKernel(reinterpret_cast<const void*>(kern), grid, block, args, lds, stream);
    const char* name = plan.ties ? "k_sweep3_packed_q" : "k_sweep3_packed";
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return ising_host::hip_failed(e, name);
    }
    return ising_host::check_launch(name);
}

// (M, E) of a packed cubic lattice added into out: two zeroed int64, or (spread) a zeroed spread set.
int launch_observables3_packed(const uint32_t* planes, int64_t L, int64_t* out, bool spread, hipStream_t s) {
    const uint64_t n = (uint64_t)L * (uint64_t)L * (uint64_t)(L / 64);
    hipLaunchKernelGGL(ising::k_observables3_packed, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, planes,
                       (uint32_t)L, (uint32_t)(L / 64), n, out, spread ? 1u : 0u);
    return ising_host::check_launch("k_observables3_packed");
}

uint64_t lanes3(int64_t L) { return (uint64_t)L * (uint64_t)L * (uint64_t)(L / 64); }

dim3 grid3(uint64_t n_lanes) { return dim3((unsigned)((n_lanes + 255) / 256)); }

}  // namespace

namespace {

// One fused sweep src -> dst: workgroups of Y own rows (W waves) plus, when Y < L, one wave with
// the two halo rows; Rz planes each.
// Planes per workgroup of the fused pass: it recomputes the planes on either side of its run, so
// it takes the tallest run (up to 128, at least 8) that still leaves ~9 waves per compute unit
// (256 CUs); option "planes3" overrides.
Shape3 shape3_fused(int64_t L) {
    Shape3 s = shape3(L);
    if (ising_host::option("planes3") > 0) return s;
    const uint32_t waves = s.W + ((int64_t)s.Y < L ? 1u : 0u);
    uint32_t Rz = 128;
    while (Rz > 8 && (L % Rz != 0 || (uint64_t)s.ystrips * (uint64_t)(L / Rz) * waves < 2304u)) Rz >>= 1;
    if (L % Rz == 0) s.Rz = Rz;
    return s;
}

int launch_sweep3_fused(const int8_t* src, int8_t* dst, int64_t L, const ising::Thresholds3& th, uint64_t seed,
                        uint32_t t, int64_t* obs, hipStream_t stream) {
    const Shape3 sh = shape3_fused(L);
    ising::Fused3Args a;
    a.src = src;
    a.dst = dst;
    a.L = (uint32_t)L;
    a.G = (uint32_t)(L / 64);
    a.Y = sh.Y;
    a.ystrips = sh.ystrips;
    a.Rz = sh.Rz;
    a.t = t;
    a.key0 = (uint32_t)seed;
    a.key1 = (uint32_t)(seed >> 32);
    a.th = th;
    a.obs = obs;
    a.xcd_remap = ising_host::xcd_remap() ? 1u : 0u;
    const bool halo = (int64_t)sh.Y < L;
    const uint32_t own = sh.W * 64u;
    const uint32_t threads = halo ? (own + 2u * a.G + 63u) / 64u * 64u : own;
    const dim3 grid(sh.ystrips * (uint32_t)(L / sh.Rz)), block(threads);
    if (ising_host::option("ties3") && sh.Rz % 2u == 0u) {
        // own rows, then the two halo rows and the two rows beyond them
        const uint32_t nq = halo ? (own + 4u * a.G + 63u) / 64u * 64u : own;
        const dim3 blockq(nq);
        const size_t lds = (size_t)(nq / 64u) * ising::kTieQueue3Bytes + 4u * nq * sizeof(uint4);
#define ISING_LAUNCH3FQ(OO, HH)                                                                            \
    do {                                                                                                   \
        if (lds > 65536) {                                                                                 \
            const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&ising::k_sweep3_fusedq<OO, HH, DD>), \
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
            if (e != hipSuccess) return ising_host::hip_failed(e, "hipFuncSetAttribute(k_sweep3_fusedq)"); \
        }                                                                                                  \
        hipLaunchKernelGGL((ising::k_sweep3_fusedq<OO, HH, DD>), grid, blockq, lds, stream, a);           \
    } while (0)
        // a wave's 4 KiB hold 4096 / L rows: direct row I/O from eight rows per wave (L <= 512) on
        if (L <= 512) {
            constexpr bool DD = true;
            if (halo) { if (obs) ISING_LAUNCH3FQ(true, true); else ISING_LAUNCH3FQ(false, true); }
            else { if (obs) ISING_LAUNCH3FQ(true, false); else ISING_LAUNCH3FQ(false, false); }
        } else {
            constexpr bool DD = false;
            if (halo) { if (obs) ISING_LAUNCH3FQ(true, true); else ISING_LAUNCH3FQ(false, true); }
            else { if (obs) ISING_LAUNCH3FQ(true, false); else ISING_LAUNCH3FQ(false, false); }
        }
#undef ISING_LAUNCH3FQ
        return ising_host::check_launch("k_sweep3_fusedq");
    }
    const size_t lds = (size_t)sh.W * 4096u + 2u * threads * sizeof(uint4);
#define ISING_LAUNCH3F(OO, HH) hipLaunchKernelGGL((ising::k_sweep3_fused<OO, HH>), grid, block, lds, stream, a)
    if (halo) { if (obs) ISING_LAUNCH3F(true, true); else ISING_LAUNCH3F(false, true); }
    else { if (obs) ISING_LAUNCH3F(true, false); else ISING_LAUNCH3F(false, false); }
#undef ISING_LAUNCH3F
    return ising_host::check_launch("k_sweep3_fused");
}

bool disjoint3(const void* x, const void* y, uint64_t bytes) {
    const uintptr_t p = reinterpret_cast<uintptr_t>(x), q = reinterpret_cast<uintptr_t>(y);
    return p + bytes <= q || q + bytes <= p;
}

}  // namespace

extern "C" {

int ising3_pack(const int8_t* spins, int64_t L, uint32_t* planes, void* stream) {
    if (!spins || !planes || !valid_L3(L) || !ising_host::aligned16(spins)) return ISING_EINVAL;
    const uint64_t n = lanes3(L);
    hipLaunchKernelGGL(ising::k_pack3, grid3(n), dim3(256), 0, (hipStream_t)stream, spins, planes, (uint32_t)L,
                       (uint32_t)(L / 64), n);
    return ising_host::check_launch("k_pack3");
}

int ising3_unpack(const uint32_t* planes, int64_t L, int8_t* spins, void* stream) {
    if (!spins || !planes || !valid_L3(L) || !ising_host::aligned16(spins)) return ISING_EINVAL;
    const uint64_t n = lanes3(L);
    hipLaunchKernelGGL(ising::k_unpack3, grid3(n), dim3(256), 0, (hipStream_t)stream, planes, spins, (uint32_t)L,
                       (uint32_t)(L / 64), n);
    return ising_host::check_launch("k_unpack3");
}

int ising3_init_packed(uint32_t* planes, int64_t L, uint64_t seed, void* stream) {
    if (!planes || !valid_L3(L)) return ISING_EINVAL;
    const uint64_t n = lanes3(L);
    hipLaunchKernelGGL(ising::k_init_packed3, grid3(n), dim3(256), 0, (hipStream_t)stream, planes, (uint32_t)L,
                       (uint32_t)(L / 64), n, (uint32_t)seed, (uint32_t)(seed >> 32));
    return ising_host::check_launch("k_init_packed3");
}

int ising3_half_sweep_packed(uint32_t* planes, int64_t L, double beta, uint64_t seed, uint64_t t, int q,
                             void* stream) {
    if (!planes || !valid_L3(L) || !ising_host::valid_beta(beta) || (q != 0 && q != 1) || t >= (uint64_t(1) << 32))
        return ISING_EINVAL;
    return launch_half_sweep3_packed(planes, L, packed3_plan(L), make_thresholds3(beta), seed, (uint32_t)t, q,
                                     nullptr, (hipStream_t)stream);
}

int ising3_sweep_packed(uint32_t* planes, int64_t L, double beta, int64_t n_sweeps, uint64_t seed,
                        uint64_t sweep_offset, int64_t* trace_ME, void* stream) {
    if (!planes || !valid_L3(L) || !ising_host::valid_beta(beta) || n_sweeps < 0 ||
        sweep_offset > (uint64_t(1) << 32) || (uint64_t)n_sweeps > (uint64_t(1) << 32) - sweep_offset)
        return ISING_EINVAL;
    const ising::Thresholds3 th = make_thresholds3(beta);
    const Packed3Plan plan = packed3_plan(L);
    hipStream_t s = (hipStream_t)stream;
    ising_host::SpreadTrace sp;
    if (trace_ME && n_sweeps > 0) {
        const int rc = sp.begin(nullptr, n_sweeps, s);
        if (rc) return rc;
    }
    for (int64_t i = 0; i < n_sweeps; ++i) {
        const uint32_t t = (uint32_t)(sweep_offset + (uint64_t)i);
        int64_t* set = nullptr;
        int rc = ISING_OK;
        if (plan.ties) {
            // the first launch of sweep i counts the lattice after sweep i - 1
            if (trace_ME && i > 0 && (rc = sp.next(trace_ME + 2 * (i - 1), 2, &set))) return rc;
            if ((rc = launch_half_sweep3_packed(planes, L, plan, th, seed, t, 1, set, s))) return rc;
            if ((rc = launch_half_sweep3_packed(planes, L, plan, th, seed, t, 0, nullptr, s))) return rc;
        } else {
            if (trace_ME && (rc = sp.next(trace_ME + 2 * i, 2, &set))) return rc;
            if ((rc = launch_half_sweep3_packed(planes, L, plan, th, seed, t, 1, nullptr, s))) return rc;
            if ((rc = launch_half_sweep3_packed(planes, L, plan, th, seed, t, 0, set, s))) return rc;
        }
    }
    if (plan.ties && trace_ME && n_sweeps > 0) {
        // the lattice after the last sweep
        int64_t* set = nullptr;
        int rc = sp.next(trace_ME + 2 * (n_sweeps - 1), 2, &set);
        if (rc) return rc;
        if ((rc = launch_observables3_packed(planes, L, set, true, s))) return rc;
    }
    return sp.fold();
}

int ising3_observables_packed(const uint32_t* planes, int64_t L, int64_t* out_ME, void* stream) {
    if (!planes || !out_ME || !valid_L3(L)) return ISING_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int rc = ising_host::zero_trace(out_ME, 2, s);
    if (rc) return rc;
    return launch_observables3_packed(planes, L, out_ME, false, s);
}

int ising3_thresholds(double beta, uint64_t out[3]) {
    if (!out || !ising_host::valid_beta(beta)) return ISING_EINVAL;
    host_thresholds3(beta, out);
    return ISING_OK;
}

int ising3_half_sweep(int8_t* spins, int64_t L, double beta, uint64_t seed, uint64_t t, int q, void* stream) {
    if (!spins || !valid_L3(L) || !ising_host::aligned16(spins) || !ising_host::valid_beta(beta) ||
        (q != 0 && q != 1) || t >= (uint64_t(1) << 32))
        return ISING_EINVAL;
    return launch_half_sweep3(spins, L, make_thresholds3(beta), seed, (uint32_t)t, q, nullptr, nullptr,
                              (hipStream_t)stream);
}

int ising3_sweep(int8_t* spins, int64_t L, double beta, int64_t n_sweeps, uint64_t seed, uint64_t sweep_offset,
                 int64_t* trace_ME, void* stream) {
    if (!spins || !valid_L3(L) || !ising_host::aligned16(spins) || !ising_host::valid_beta(beta) || n_sweeps < 0 ||
        sweep_offset > (uint64_t(1) << 32) || (uint64_t)n_sweeps > (uint64_t(1) << 32) - sweep_offset)
        return ISING_EINVAL;
    const ising::Thresholds3 th = make_thresholds3(beta);
    hipStream_t s = (hipStream_t)stream;
    for (int64_t i = 0; i < n_sweeps; ++i) {
        const uint32_t t = (uint32_t)(sweep_offset + (uint64_t)i);
        int64_t* slot = trace_ME ? trace_ME + 2 * i : nullptr;
        int rc = launch_half_sweep3(spins, L, th, seed, t, 1, nullptr, slot, s);  // white (zeroes the slot)
        if (rc) return rc;
        rc = launch_half_sweep3(spins, L, th, seed, t, 0, slot, nullptr, s);      // black (+ M, E)
        if (rc) return rc;
    }
    return ISING_OK;
}

int ising3_sweep_fused(int8_t* spins, int8_t* scratch, int64_t L, double beta, int64_t n_sweeps, uint64_t seed,
                       uint64_t sweep_offset, int64_t* trace_ME, void* stream) {
    if (!spins || !scratch || !valid_L3(L) || !ising_host::aligned16(spins) || !ising_host::aligned16(scratch) ||
        !ising_host::valid_beta(beta) || n_sweeps < 0 || sweep_offset > (uint64_t(1) << 32) ||
        (uint64_t)n_sweeps > (uint64_t(1) << 32) - sweep_offset ||
        !disjoint3(spins, scratch, (uint64_t)L * (uint64_t)L * (uint64_t)L))
        return ISING_EINVAL;
    const ising::Thresholds3 th = make_thresholds3(beta);
    hipStream_t s = (hipStream_t)stream;
    int64_t i = 0;
    if (n_sweeps & 1) {  // an odd count: the first sweep in place, so that the pairs end in `spins`
        const int rc = ising3_sweep(spins, L, beta, 1, seed, sweep_offset, trace_ME, stream);
        if (rc) return rc;
        i = 1;
    }
    if (trace_ME) {
        const int rc = ising_host::zero_trace(trace_ME + 2 * i, 2 * (n_sweeps - i), s);
        if (rc) return rc;
    }
    for (; i < n_sweeps; i += 2) {
        const uint32_t t = (uint32_t)(sweep_offset + (uint64_t)i);
        int rc = launch_sweep3_fused(spins, scratch, L, th, seed, t, trace_ME ? trace_ME + 2 * i : nullptr, s);
        if (rc) return rc;
        rc = launch_sweep3_fused(scratch, spins, L, th, seed, t + 1, trace_ME ? trace_ME + 2 * i + 2 : nullptr, s);
        if (rc) return rc;
    }
    return ISING_OK;
}

int ising3_sweep_fused_step(const int8_t* src, int8_t* dst, int64_t L, double beta, uint64_t seed, uint64_t t,
                            int64_t* out_ME, void* stream) {
    if (!src || !dst || !valid_L3(L) || !ising_host::aligned16(src) || !ising_host::aligned16(dst) ||
        !ising_host::valid_beta(beta) || t >= (uint64_t(1) << 32) ||
        !disjoint3(src, dst, (uint64_t)L * (uint64_t)L * (uint64_t)L))
        return ISING_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (out_ME) {
        const int rc = ising_host::zero_trace(out_ME, 2, s);
        if (rc) return rc;
    }
    return launch_sweep3_fused(src, dst, L, make_thresholds3(beta), seed, (uint32_t)t, out_ME, s);
}

int ising3_observables(const int8_t* spins, int64_t L, int64_t* out_ME, void* stream) {
    if (!spins || !out_ME || !valid_L3(L) || !ising_host::aligned16(spins)) return ISING_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int rc = ising_host::zero_trace(out_ME, 2, s);
    if (rc) return rc;
    const uint32_t G = (uint32_t)(L / 64);
    const uint64_t n_lanes = (uint64_t)L * (uint64_t)L * G;
    hipLaunchKernelGGL(ising::k_observables3, dim3((unsigned)((n_lanes + 255) / 256)), dim3(256), 0, s, spins,
                       (uint32_t)L, G, n_lanes, out_ME);
    return ising_host::check_launch("k_observables3");
}

}  // extern "C"
