// rows.hpp — device building blocks shared by the sweep kernels (square and cubic lattices).
//
// A lane owns a "group": 64 consecutive columns of one row, i.e. 32 sites of each colour.  Rows
// move between HBM and registers with coalesced 16-byte loads and stores regrouped per lane
// through LDS, and are reduced to bit words (one bit per site, 32 same-colour sites per word in
// "site order", the bit position their uniform uses in each Philox word).  The Metropolis test
// compares each site's uniform with its threshold bit plane by bit plane, four planes per Philox
// block, until no site of the wave is still tied (Sec. 3.2, Algorithm 1: uniform below the
// acceptance ratio).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "philox.hpp"

namespace ising {

// ------------------------------------------------------------------------------------------
// Bit-word helpers.  "Site order": site i (0..31) of a group sits at bit p(i) =
// 8 * (0, 2, 1, 3)[i & 3] + (i >> 2), the bit position its uniform uses in each Philox word.

struct Row {
    uint32_t d[16];  // 64 bytes = one group of one row; dword k holds columns 4k .. 4k + 3
};

__device__ __forceinline__ uint32_t perm(uint32_t s0, uint32_t s1, uint32_t sel) {
    return __builtin_amdgcn_perm(s0, s1, sel);
}

// (a & b) | c as one v_bitop3_b32 (truth table over a = 0xF0, b = 0xCC, c = 0xAA)
__device__ __forceinline__ uint32_t and_or3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0xEA);
}

__device__ __forceinline__ void load_row(Row& row, const int8_t* p) {
    const uint4* v = reinterpret_cast<const uint4*>(p);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint4 x = v[i];
        row.d[4 * i + 0] = x.x;
        row.d[4 * i + 1] = x.y;
        row.d[4 * i + 2] = x.z;
        row.d[4 * i + 3] = x.w;
    }
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void store_row(int8_t* p, const Row& row, bool streaming) {
    u32x4* v = reinterpret_cast<u32x4*>(p);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const u32x4 x = {row.d[4 * i], row.d[4 * i + 1], row.d[4 * i + 2], row.d[4 * i + 3]};
        if (streaming) __builtin_nontemporal_store(x, v + i);
        else v[i] = x;
    }
}

// ---- Coalesced row I/O through LDS.  When a wave's 64 lanes own 64 consecutive groups of
// one row (4 KiB), loading "64 contiguous bytes per lane" wastes most of every memory
// instruction.  Instead lane l moves 16-byte chunks l, l + 64, l + 128, l + 192 of the wave's
// row segment (each instruction covers 1 KiB contiguous) and the bytes are regrouped per lane
// through a 4 KiB per-wave LDS buffer.  Chunk c belongs to lane c / 4, quarter c % 4, and is
// kept in LDS slot 4 (c / 4) + ((c % 4 + c / 8) mod 4): any 8 consecutive lanes then touch 8
// distinct 16-byte bank groups on both the write and the read side.
__device__ __forceinline__ uint32_t lds_slot(uint32_t owner, uint32_t quarter) {
    return 4u * owner + ((quarter + (owner >> 1)) & 3u);
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// raw: this lane's four coalesced chunks (chunk l + 64 k in raw.d[4k .. 4k + 3]).
__device__ __forceinline__ void load_row_coalesced(Row& raw, const int8_t* seg, uint32_t lane) {
    const uint4* v = reinterpret_cast<const uint4*>(seg) + lane;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint4 x = v[64 * k];
        raw.d[4 * k + 0] = x.x;
        raw.d[4 * k + 1] = x.y;
        raw.d[4 * k + 2] = x.z;
        raw.d[4 * k + 3] = x.w;
    }
}

// coalesced chunks -> this lane's own 64 bytes
__device__ __forceinline__ void regroup_to_owner(Row& row, const Row& raw, uint4* lds, uint32_t lane) {
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
        const uint32_t c = lane + 64u * k;
        lds[lds_slot(c >> 2, c & 3u)] = make_uint4(raw.d[4 * k], raw.d[4 * k + 1], raw.d[4 * k + 2], raw.d[4 * k + 3]);
    }
    wave_lds_sync();
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
        const uint4 x = lds[lds_slot(lane, q)];
        row.d[4 * q + 0] = x.x;
        row.d[4 * q + 1] = x.y;
        row.d[4 * q + 2] = x.z;
        row.d[4 * q + 3] = x.w;
    }
    wave_lds_sync();
}

// this lane's own 64 bytes -> coalesced stores of the wave's row segment
__device__ __forceinline__ void store_row_coalesced(int8_t* seg, const Row& row, uint4* lds, uint32_t lane,
                                                    bool streaming) {
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q)
        lds[lds_slot(lane, q)] = make_uint4(row.d[4 * q], row.d[4 * q + 1], row.d[4 * q + 2], row.d[4 * q + 3]);
    wave_lds_sync();
    u32x4* v = reinterpret_cast<u32x4*>(seg) + lane;
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
        const uint32_t c = lane + 64u * k;
        const uint4 x = lds[lds_slot(c >> 2, c & 3u)];
        const u32x4 y = {x.x, x.y, x.z, x.w};
        if (streaming) __builtin_nontemporal_store(y, v + 64 * k);
        else v[64 * k] = y;
    }
    wave_lds_sync();
}

// ---- Row I/O of a column band: a wave whose 64 lanes own 64 consecutive groups of a row modulo the
// row length G >= 64 (a band can wrap round the torus seam, so the groups need not be contiguous in
// memory).  Lane l moves the 16-byte chunks c = l + 64 k of the band's 64 groups: chunk c is quarter
// c % 4 of the band's group c / 4 = l / 4 + 16 k, i.e. of row group (gbase + 16 k) mod G with gbase =
// the row group of band group l / 4.  The chunks are regrouped per lane through the wave's 4 KiB of
// LDS exactly as for a contiguous segment.
__device__ __forceinline__ uint32_t band_chunk_offset(uint32_t gbase, uint32_t k, uint32_t G, uint32_t lane) {
    uint32_t gk = gbase + 16u * k;  // < G + 48 <= 2G
    gk = gk >= G ? gk - G : gk;
    return gk * 64u + (lane & 3u) * 16u;
}

__device__ __forceinline__ void load_row_chunks(Row& raw, const int8_t* row, uint32_t gbase, uint32_t G,
                                                uint32_t lane) {
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
        const uint4 x = *reinterpret_cast<const uint4*>(row + band_chunk_offset(gbase, k, G, lane));
        raw.d[4 * k + 0] = x.x;
        raw.d[4 * k + 1] = x.y;
        raw.d[4 * k + 2] = x.z;
        raw.d[4 * k + 3] = x.w;
    }
}

// this lane's own 64 bytes -> the band's chunks; only the chunks of band groups 1 .. n_own are stored
__device__ __forceinline__ void store_row_chunks(int8_t* row, const Row& own, uint4* lds, uint32_t lane,
                                                 uint32_t gbase, uint32_t G, uint32_t n_own, bool streaming) {
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q)
        lds[lds_slot(lane, q)] = make_uint4(own.d[4 * q], own.d[4 * q + 1], own.d[4 * q + 2], own.d[4 * q + 3]);
    wave_lds_sync();
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
        const uint32_t c = lane + 64u * k;
        const uint4 x = lds[lds_slot(c >> 2, c & 3u)];
        const u32x4 y = {x.x, x.y, x.z, x.w};
        u32x4* v = reinterpret_cast<u32x4*>(row + band_chunk_offset(gbase, k, G, lane));
        const uint32_t owner = (lane >> 2) + 16u * k;
        if (owner >= 1u && owner <= n_own) {
            if (streaming) __builtin_nontemporal_store(y, v);
            else *v = y;
        }
    }
    wave_lds_sync();
}

// Workgroups are dispatched to the eight XCDs round robin (block b runs on XCD b mod 8).
// Renumbering them so that each XCD receives one contiguous range of logical blocks keeps
// neighbouring row strips, which read each other's boundary rows, inside one L2.
__device__ __forceinline__ uint32_t logical_block(uint32_t b, uint32_t nb, bool remap) {
    if (!remap) return b;
    const uint32_t x = b & 7u, i = b >> 3, per = nb >> 3, rem = nb & 7u;
    return x * per + (x < rem ? x : rem) + i;
}

// Sign bits (1 = spin -1) of the 32 sites at columns of parity OFF, in site order.
// A +-1 byte is 0x01 or 0xFF, so bits 1..7 of the byte all equal its sign.
template <int OFF>
__device__ __forceinline__ uint32_t site_bits(const Row& row) {
    // bytes of the compact word: (site 4k, site 4k+2, site 4k+1, site 4k+3)
    constexpr uint32_t sel = OFF | ((4 + OFF) << 8) | ((OFF + 2) << 16) | ((6 + OFF) << 24);
    uint32_t acc = (perm(row.d[1], row.d[0], sel) >> 1) & 0x01010101u;
#pragma unroll
    for (int k = 1; k < 8; ++k) acc |= perm(row.d[2 * k + 1], row.d[2 * k], sel) & (0x01010101u << k);
    return acc;
}

// S[p(i)] = y[p(i + 1)] for i < 31, S[p(31)] = bit0 (site 0 of the next group).
__device__ __forceinline__ uint32_t shift_next(uint32_t y, uint32_t bit0) {
    const uint32_t top = ((y >> 1) & 0x7Fu) | (bit0 << 7);
    return perm(top, y, 0x04010302u);
}

// S[p(i)] = y[p(i - 1)] for i > 0, S[p(0)] = bit31 (site 31 of the previous group).
__device__ __forceinline__ uint32_t shift_prev(uint32_t y, uint32_t bit31) {
    const uint32_t low = ((y >> 23) & 0xFEu) | bit31;
    return perm(y, low, 0x05040600u);
}

// ---- Half groups.  A row whose length L is an odd multiple of 32 ends in a group of 32 columns:
// 16 sites of each colour, sites 0 .. 15, i.e. bits 0 .. 3 of every byte in site order.
constexpr uint32_t kHalfSites = 0x0F0F0F0Fu;

// shift_next for a half group: S[p(i)] = y[p(i + 1)] for i < 15, S[p(15)] = bit0 (site 0 of the next
// group); the bits of sites 16 .. 31 are zero.
__device__ __forceinline__ uint32_t shift_next_half(uint32_t y, uint32_t bit0) {
    const uint32_t top = ((y >> 1) & 0x07u) | (bit0 << 3);
    return perm(top, y, 0x04010302u) & kHalfSites;
}

// The bit of a group word's last site: site 31 (bit 31), or site 15 (bit 27) of a half group.
__device__ __forceinline__ uint32_t last_site_bit(uint32_t y, bool half) { return half ? (y >> 27) & 1u : y >> 31; }

// A half group's 32 bytes; the other half of the row buffer holds +1 spins (0x01), which no decision
// reads (every result is masked with kHalfSites).
__device__ __forceinline__ void load_row_half(Row& row, const int8_t* p) {
    const uint4* v = reinterpret_cast<const uint4*>(p);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const uint4 x = v[i];
        row.d[4 * i + 0] = x.x;
        row.d[4 * i + 1] = x.y;
        row.d[4 * i + 2] = x.z;
        row.d[4 * i + 3] = x.w;
    }
#pragma unroll
    for (int k = 8; k < 16; ++k) row.d[k] = 0x01010101u;
}

__device__ __forceinline__ void store_row_half(int8_t* p, const Row& row) {
    uint4* v = reinterpret_cast<uint4*>(p);
    v[0] = make_uint4(row.d[0], row.d[1], row.d[2], row.d[3]);
    v[1] = make_uint4(row.d[4], row.d[5], row.d[6], row.d[7]);
}

// Flip the colour-OFF bytes of `row` whose site bit is set in F.  The two sites of dword
// 2k + h sit at bits k + 8h and k + 8h + 16; shifting them to bits 15 and 31 lets the
// sign-extending selectors 8 and 9 of v_perm produce 0xFF at exactly those bytes.
template <int OFF>
__device__ __forceinline__ void apply_flips(Row& row, uint32_t F) {
    constexpr uint32_t sel = OFF == 0 ? 0x0C090C08u : 0x090C080Cu;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t m = perm(0u, F << (15 - k - 8 * h), sel);
            row.d[2 * k + h] ^= m & 0xFEFEFEFEu;  // 0x01 <-> 0xFF
        }
    }
}

__device__ __forceinline__ bool wave_any(bool v) { return __builtin_amdgcn_ballot_w64(v) != 0; }

// Metropolis thresholds of one launch (uniform): a site with a anti-aligned neighbours has
// s = 4 - 2a; a >= 2 always flips, a = 1 compares with T_2, a = 0 with T_4.
struct Thresholds {
    uint32_t t2, t4;      // low 32 bits of T_2, T_4
    uint32_t f2, f4;      // all ones when T_s = 2^32 (always accept), else zero
    uint32_t blocks;        // Philox blocks (4 bit planes each) that can decide: 8, or 4 when
                            // both thresholds are multiples of 2^16 (16-bit uniforms)
};

// The four bit planes of one Philox block (planes 4m .. 4m + 3) against the thresholds: a tied site
// whose uniform has 0 where its threshold has 1 is accepted (x < T), one that differs the other way
// is decided against, one that agrees stays tied.
// OR3: the accepted sites of each two planes enter acc through one three-input v_bitop3 instead of
// the v_or3_b32 the compiler forms from the same ors; gfx950 issues v_bitop3_b32 at twice the rate of
// v_or3_b32.  The packed half-sweep, bound by issue, runs 1.2-1.6% faster with it; the two-sweep passes,
// bound by latency, measured no gain.
template <bool OR3 = false>
__device__ __forceinline__ void compare_planes(uint32_t& acc, uint32_t& tied, uint32_t sel2, const Words4& blk,
                                               const Thresholds& th, uint32_t m) {
    const uint32_t planes[4] = {blk.w0, blk.w1, blk.w2, blk.w3};
    uint32_t won[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const uint32_t k = 4u * m + (uint32_t)w;
        // the site's threshold bit is bit 31 - k of T_4 (m4), flipped on sel2 where T_2 differs (d); the
        // uniform masks enter one at a time (a vector instruction reads at most one scalar register):
        // diff = x ^ m4 ^ (sel2 & d) = x ^ threshold bit.  (Branching on the uniform bits measured slower.)
        const uint32_t m4 = 0u - ((th.t4 >> (31u - k)) & 1u);
        const uint32_t d = 0u - (((th.t2 ^ th.t4) >> (31u - k)) & 1u);
        const uint32_t x = planes[w];
        // four instructions: the compiler would otherwise fold the masks back into five
        const uint32_t diff = __builtin_amdgcn_bitop3_b32(x ^ m4, sel2, d, 0x78);  // a ^ (b & c)
        won[w] = __builtin_amdgcn_bitop3_b32(tied, diff, x, 0x40);  // differs with x = 0: threshold bit 1, x < T
        if (!OR3) acc |= won[w];
        tied = __builtin_amdgcn_bitop3_b32(tied, diff, 0u, 0x30);  // a & ~b
    }
    if (OR3) {
        acc = __builtin_amdgcn_bitop3_b32(acc, won[0], won[1], 0xFE);  // a | b | c
        acc = __builtin_amdgcn_bitop3_b32(acc, won[2], won[3], 0xFE);
    }
}

// Exact x < T for every site in sel2 (threshold T_2) or sel4 (T_4), bit plane by bit plane.
// Returns the accepted sites.  Planes come four per Philox block with counter
// (g, r, t, 2m + q), plane k = 4m + w is bit 31 - k of each site's uniform.
__device__ __forceinline__ uint32_t accept_mask(uint32_t sel2, uint32_t sel4, const Thresholds& th,
                                                uint32_t g, uint32_t r, uint32_t t, uint32_t q,
                                                uint32_t key0, uint32_t key1) {
    uint32_t acc = (sel2 & th.f2) | (sel4 & th.f4);
    sel2 &= ~th.f2;
    sel4 &= ~th.f4;
    uint32_t tied = sel2 | sel4;
    // sites outside sel2 are compared with T_4 below; make sure only tied ones matter
#pragma unroll 1
    for (uint32_t m = 0; m < th.blocks; ++m) {
        // a site still tied after the last deciding plane has x >= T (the remaining bits of T
        // are zero), so it is rejected
        if (!wave_any(tied != 0)) break;
        compare_planes(acc, tied, sel2, philox4x32_10(g, r, t, 2u * m + q, key0, key1), th, m);
    }
    return acc;
}

struct Counts {
    uint32_t anti;  // anti-aligned bonds seen from this colour's sites after the update
    uint32_t neg;   // spins equal to -1 in the rows processed
};

// Sum over the 64 lanes of a wave (every lane active), returned to every lane.  Lane shifts (DPP)
// instead of LDS permutes: prefix sums within each row of 16 lanes (row_shr by 1, 2, 3 of the value,
// then by 4 and 8 on the upper banks), rows 1 and 3 add the last lane of the row before (row_bcast:15),
// rows 2 and 3 that of row 1 (row_bcast:31); lane 63 then holds the total.  Masked-off lanes and lanes
// shifted in from outside a row take 0.
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
    uint32_t x = v;
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true);  // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true);  // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x113, 0xf, 0xf, true);  // row_shr:3
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xe, true);  // row_shr:4, lanes 4..15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xc, true);  // row_shr:8, lanes 8..15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, true);  // row_bcast:15, rows 1, 3
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, true);  // row_bcast:31, rows 2, 3
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// Block-level sum of (anti, neg) -> one pair of 64-bit atomics per block.
// sites_per_lane: sites each active lane covered; bonds_per_site: 2 on the square lattice, 3 on
// the cubic one (anti counts every anti-aligned bond once).
__device__ __forceinline__ void block_accumulate(int64_t* out, uint32_t anti, uint32_t neg, uint32_t active,
                                                 uint32_t sites_per_lane, uint32_t bonds_per_site = 2) {
    __shared__ uint32_t red[3][16];
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    anti = wave_sum(anti);
    neg = wave_sum(neg);
    active = wave_sum(active);
    if (lane == 0) { red[0][wave] = anti; red[1][wave] = neg; red[2][wave] = active; }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t A = 0, Nn = 0, act = 0;
        for (uint32_t w = 0; w < blockDim.x / 64u; ++w) { A += red[0][w]; Nn += red[1][w]; act += red[2][w]; }
        const int64_t sites = (int64_t)act * sites_per_lane;
        const int64_t M = sites - 2 * (int64_t)Nn;            // sum of spins
        const int64_t E = 2 * (int64_t)A - (int64_t)bonds_per_site * sites;  // #anti - #aligned
        atomicAdd(reinterpret_cast<unsigned long long*>(out), (unsigned long long)M);
        atomicAdd(reinterpret_cast<unsigned long long*>(out + 1), (unsigned long long)E);
    }
}

// ---- Spread accumulation of (M, E).  Atomics of every workgroup of a launch on the same two words
// queue at one memory channel as the workgroups end.  A traced launch of the sweep loops adds into
// one of kSpreadLines 128-byte lines of a set (the line chosen by workgroup) instead, and a later
// one-wave-per-set kernel sums each set's lines into the trace and clears them.
constexpr uint32_t kSpreadLines = 64;
constexpr uint32_t kSpreadLineWords = 16;                              // int64 per 128-byte line
constexpr uint32_t kSpreadSetWords = kSpreadLines * kSpreadLineWords;  // one launch's set: 8 KiB

__device__ __forceinline__ int64_t* spread_line(int64_t* set, uint32_t block) {
    return set + (size_t)(block % kSpreadLines) * kSpreadLineWords;
}

struct RowBits {
    uint32_t e, o;  // sign bits of the even / odd columns of one group of one row, site order
};

__device__ __forceinline__ RowBits row_bits(const Row& row) { return RowBits{site_bits<0>(row), site_bits<1>(row)}; }

// inverse of row_bits: +1 -> 0x01, -1 -> 0xFF
__device__ __forceinline__ void bits_to_row(Row& row, const RowBits& b) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t sh = 15 - k - 8 * h;
            row.d[2 * k + h] = perm(b.o << sh, b.e << sh, 0x0B090A08u) | 0x01010101u;
        }
    }
}

// ---- Tie queue.  A wave decides a word's sites with as many Philox blocks as its least
// decided site needs, though 15 of 16 sites are decided by the first block.  Where a lane has
// several independent words to decide (rows of one colour update, or updates of one step that do
// not read each other), each word takes its first two blocks at once and the words still holding
// tied sites go to a per-wave queue in LDS; the wave then settles the queue one word per lane, so
// the later planes cost a block per 64 queued words instead of one per word position.

// Per-wave LDS of a tie queue (5 KiB).  Entry j = one word with sites still tied: those sites,
// the ones of them compared with T_2, the Philox row, and update | lane << 2 | group << 8.
// res[lane] = the sites of the lane's updates 0 .. 3 that the queue accepted (zeroed before the
// pushes).
struct TieQueue {
    uint32_t* task;  // [4][256]: tied, tied & sel2, row, meta
    uint4* res;      // [64]
};
constexpr uint32_t kTieQueueBytes = 256u * 16u + 64u * 16u;

// Appends the lane's word to the queue if it has tied sites (n = entries so far, uniform).
__device__ __forceinline__ void tq_push(const TieQueue& q, uint32_t& n, uint32_t tied, uint32_t sel2, uint32_t row,
                                        uint32_t meta) {
    const uint64_t B = __builtin_amdgcn_ballot_w64(tied != 0u);
    if (tied != 0u) {
        const uint32_t pos =
            n + __builtin_amdgcn_mbcnt_hi((uint32_t)(B >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)B, 0u));
        q.task[pos] = tied;
        q.task[256u + pos] = sel2 & tied;
        q.task[512u + pos] = row;
        q.task[768u + pos] = meta;
    }
    n += (uint32_t)__builtin_popcountll(B);
}

// Settles the n queued words (n <= 256), one per lane, with the planes of blocks 2 onwards.  The
// uniform of a word of update u has sweep t + u / 2 and colour 1 - u % 2 when QC < 0 (the
// two-sweep walk), sweep t and colour QC otherwise.
template <int QC>
__device__ __forceinline__ void tq_settle(const TieQueue& q, uint32_t n, const Thresholds& th, uint32_t t,
                                          uint32_t key0, uint32_t key1, uint32_t lane) {
    wave_lds_sync();
#pragma unroll 1
    for (uint32_t b = 0; b < n; b += 64u) {
        const uint32_t j = b + lane;
        const bool have = j < n;
        uint4 tk = make_uint4(0u, 0u, 0u, 0u);
        if (have) tk = make_uint4(q.task[j], q.task[256u + j], q.task[512u + j], q.task[768u + j]);
        const uint32_t u = tk.w & 3u, src = (tk.w >> 2) & 63u, g = tk.w >> 8;
        const uint32_t tu = QC < 0 ? t + (u >> 1) : t, qu = QC < 0 ? (u & 1u) ^ 1u : (uint32_t)QC;
        uint32_t acc = 0u, tied = tk.x;
#pragma unroll 1
        for (uint32_t m = 2; m < th.blocks; ++m) {
            if (!wave_any(tied != 0u)) break;
            compare_planes(acc, tied, tk.y, philox4x32_10(g, tk.z, tu, 2u * m + qu, key0, key1), th, m);
        }
        if (have) reinterpret_cast<uint32_t*>(q.res)[4u * src + u] = acc;
    }
    wave_lds_sync();
}

__device__ __forceinline__ void workgroup_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}


}  // namespace ising
