// rd_device.h -- device helpers shared by every kernel file (gfx950, wave64).
//
// The per-voxel update lives here once (rd_update) so that every kernel variant
// (block edge 4 or 8, batched, graph-replayed, solver, adjoint) performs the same
// FP32 operations in the same order and therefore gives bitwise-identical results.
// Kernel files are compiled with -ffp-contract=off; fused multiply-adds are
// explicit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rd_internal.h"

// ---- storage types ----------------------------------------------------------
// FP32 storage, BF16 storage (uint16 bit pattern, round-to-nearest-even on store)
// and FP16 storage (IEEE binary16, RNE on store).  Arithmetic is always FP32.
struct bf16_t {
    uint16_t bits;
};

__device__ __forceinline__ float rd_ld(const float *p, int64_t i) { return p[i]; }
__device__ __forceinline__ float rd_ld(const bf16_t *p, int64_t i)
{
    return __uint_as_float((uint32_t)p[i].bits << 16);
}
__device__ __forceinline__ float rd_ld(const _Float16 *p, int64_t i) { return (float)p[i]; }

// BF16 round to nearest even on the upper 16 bits; NaN stays NaN (quiet bit set).
__device__ __forceinline__ uint16_t bf16_rne(float v)
{
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// FP32 fields are streamed (written once per step, read by the next step), so their
// stores are nontemporal (measured faster on the 512^3 soil volume).
__device__ __forceinline__ void rd_st(float *p, int64_t i, float v) { __builtin_nontemporal_store(v, p + i); }
__device__ __forceinline__ void rd_st(bf16_t *p, int64_t i, float v) { p[i].bits = bf16_rne(v); }
__device__ __forceinline__ void rd_st(_Float16 *p, int64_t i, float v) { p[i] = (_Float16)v; }
// The value a round-to-nearest store into T holds when read back.
template <typename T> __device__ __forceinline__ float rd_round(float v);
template <> __device__ __forceinline__ float rd_round<float>(float v) { return v; }
template <> __device__ __forceinline__ float rd_round<bf16_t>(float v)
{
    return __uint_as_float((uint32_t)bf16_rne(v) << 16);
}
template <> __device__ __forceinline__ float rd_round<_Float16>(float v) { return (float)(_Float16)v; }

// Plain (cached) store with round to nearest, for vectors that are read again soon
// (the solver's).
__device__ __forceinline__ void rd_st_keep(float *p, int64_t i, float v) { p[i] = v; }
__device__ __forceinline__ void rd_st_keep(bf16_t *p, int64_t i, float v) { p[i].bits = bf16_rne(v); }
__device__ __forceinline__ void rd_st_keep(_Float16 *p, int64_t i, float v) { p[i] = (_Float16)v; }

// ---- predicated loads ---------------------------------------------------------
// A kernel that skips inactive voxels loads raw storage words under a predicate
// (ld_raw, 0 where the predicate is false) and converts them to FP32 only after all of
// its loads are issued (from_raw).  The conversion of BF16 / FP16 words is opaque
// inline asm: written as plain C it is folded into each predicated load's branch,
// which then waits for its own load, so the loads would no longer overlap.
__device__ __forceinline__ float ld_raw(const float *p, int64_t i, bool pred)
{
    return pred ? p[i] : 0.0f;
}
__device__ __forceinline__ uint32_t ld_raw(const bf16_t *p, int64_t i, bool pred)
{
    return pred ? (uint32_t)p[i].bits : 0u;
}
__device__ __forceinline__ uint32_t ld_raw(const _Float16 *p, int64_t i, bool pred)
{
    return pred ? (uint32_t)__builtin_bit_cast(uint16_t, p[i]) : 0u;
}
// unpredicated forms, for several loads under one predicate
__device__ __forceinline__ float ld_raw(const float *p, int64_t i) { return p[i]; }
__device__ __forceinline__ uint32_t ld_raw(const bf16_t *p, int64_t i) { return (uint32_t)p[i].bits; }
__device__ __forceinline__ uint32_t ld_raw(const _Float16 *p, int64_t i)
{
    return (uint32_t)__builtin_bit_cast(uint16_t, p[i]);
}
template <typename T> struct RawOf { typedef uint32_t type; };
template <> struct RawOf<float> { typedef float type; };

template <typename T> __device__ __forceinline__ float from_raw(typename RawOf<T>::type r);
template <> __device__ __forceinline__ float from_raw<float>(float r) { return r; }
template <> __device__ __forceinline__ float from_raw<bf16_t>(uint32_t r)
{
    float f;  // BF16 is the upper half of an FP32 pattern
    asm("v_lshlrev_b32 %0, 16, %1" : "=v"(f) : "v"(r));
    return f;
}
template <> __device__ __forceinline__ float from_raw<_Float16>(uint32_t r)
{
    float f;  // exact FP16 -> FP32 conversion of the low half
    asm("v_cvt_f32_f16 %0, %1" : "=v"(f) : "v"(r));
    return f;
}

// ---- store granularity ------------------------------------------------------
// The step kernels write a slot when any voxel of its aligned sector of
// RD_STORE_SECTOR bytes is active; the inactive slots of such a sector store the 0
// they already hold.  Sectors without an active voxel are never written, and the
// memory side only ever sees whole sectors (no partially written ones).
#ifndef RD_STORE_SECTOR
#define RD_STORE_SECTOR 128
#endif
// W: a 64-slot activity word, bit: the slot's bit in it (slots are consecutive in
// memory within the word).
template <typename T>
__device__ __forceinline__ bool sector_active(uint64_t W, int bit)
{
    // slots per sector, at most the 64 slots of one activity word
    constexpr int V = RD_STORE_SECTOR / (int)sizeof(T) < 64 ? RD_STORE_SECTOR / (int)sizeof(T) : 64;
    static_assert(V >= 1 && (V & (V - 1)) == 0, "sector of 1..64 slots");
    if constexpr (V == 64) return W != 0ull;
    else return ((W >> (bit & ~(V - 1))) & ((1ull << V) - 1ull)) != 0ull;
}

// Wave-level forms for the one-wave-per-block kernels, where slot bit l of a plane
// word belongs to lane l and the word is wave-uniform: lane_bit gives lane l bit l of
// W (the word becomes the execution mask; no per-lane shift), sector_lanes the
// uniform mask of the lanes whose sector holds an active slot (scalar ops only).
__device__ __forceinline__ bool lane_bit(uint64_t W) { return __builtin_amdgcn_inverse_ballot_w64(W); }
template <typename T>
__device__ __forceinline__ uint64_t sector_lanes(uint64_t W)
{
    constexpr int V = RD_STORE_SECTOR / (int)sizeof(T) < 64 ? RD_STORE_SECTOR / (int)sizeof(T) : 64;
    if constexpr (V == 64) {
        return W != 0ull ? ~0ull : 0ull;
    } else {
        constexpr uint64_t ONE = (1ull << V) - 1ull;
        uint64_t m = 0ull;
#pragma unroll
        for (int s = 0; s < 64; s += V) m |= ((W >> s) & ONE) != 0ull ? ONE << s : 0ull;
        return m;
    }
}

// ---- stochastic rounding --------------------------------------------------
// 32-bit finaliser of MurmurHash3 (Appleby): a bijective avalanche mix, used as
// a counter-based generator keyed by (slot, species, step, seed).
__device__ __forceinline__ uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x85ebca6bu;
    x ^= x >> 13;
    x *= 0xc2b2ae35u;
    x ^= x >> 16;
    return x;
}

// The random bits of a store come in layers so that a kernel spends little per voxel:
// a key per (step, seed), wave-uniform; a column word from the key and the voxel's
// (x, y) column in its box and a plane word from the key and its z plane (so the bits
// do not depend on the block layout, and a kernel that walks a z-column hashes the
// column once and each plane once per wave); their XOR, finalised by one
// xorshift-multiply-xorshift round (the first half of the MurmurHash3 finaliser), is the
// voxel's 32-bit word; 16 bits per species out of it (species 2 and 3 mix the voxel word
// once more).  For a fixed voxel the word is a bijection of the uniformly distributed
// column-plane XOR, so its bits are uniform over the steps' keys.
__device__ __forceinline__ uint32_t sr_key(uint32_t step, uint32_t seed)
{
    return mix32(step ^ mix32(seed + 0x9e3779b9u));
}
__device__ __forceinline__ uint32_t sr_column(const GeomInfo &g, int gx, int gy, uint32_t key)
{
    return mix32(((uint32_t)gy * (uint32_t)g.nx + (uint32_t)gx) ^ key);
}
__device__ __forceinline__ uint32_t sr_plane(int gz, uint32_t key)
{
    return mix32((uint32_t)gz ^ mix32(key ^ 0x3c6ef372u));
}
__device__ __forceinline__ uint32_t sr_combine(uint32_t column, uint32_t plane)
{
    uint32_t x = column ^ plane;
    x ^= x >> 16;
    x *= 0x85ebca6bu;
    x ^= x >> 13;
    return x;
}
__device__ __forceinline__ uint32_t sr_voxel(const GeomInfo &g, int gx, int gy, int gz, uint32_t key)
{
    return sr_combine(sr_column(g, gx, gy, key), sr_plane(gz, key));
}
__device__ __forceinline__ uint32_t sr_species(uint32_t h, int species)
{
    const uint32_t w = species < 2 ? h : mix32(h ^ 0x165667b1u);
    return (species & 1) ? (w >> 16) : (w & 0xffffu);
}

// Store with stochastic rounding: round up with probability equal to the distance
// from the lower neighbour, in units of the storage spacing (unbiased on average).
// Both forms add random bits below the cut of the FP32 pattern and truncate there, so
// the magnitude rounds up exactly when the added bits carry across the cut; no branches.
__device__ __forceinline__ uint16_t bf16_sr(float v, uint32_t rnd)
{
    // BF16 is the upper half of the FP32 pattern: 16 random bits below the cut round the
    // magnitude up with probability (low bits) / 2^16.  Infinities keep their zero low
    // bits' pattern above the cut; a NaN stays a (quiet) NaN.
    const uint32_t u = __float_as_uint(v);
    const bool nan = (u & 0x7fffffffu) > 0x7f800000u;
    return nan ? (uint16_t)((u >> 16) | 0x40u) : (uint16_t)((u + (rnd & 0xffffu)) >> 16);
}

__device__ __forceinline__ _Float16 f16_sr(float v, uint32_t rnd)
{
    // FP16 keeps 10 mantissa bits down to 2^-14 (13 FP32 bits below its cut) and a fixed
    // spacing of 2^-24 below (d = 126 - biased exponent bits below the cut, up to 23);
    // d random bits (the 16 given, shifted into the top of the d) are added to the
    // magnitude's pattern and the low d bits cleared, which leaves a multiple of the FP16
    // spacing (a carry into the exponent is the next power of two).  Below 2^-24 the
    // result is 2^-24 with probability |v| / 2^-24, else 0.  Infinities and NaNs convert
    // as they are.
    const uint32_t u = __float_as_uint(v);
    const uint32_t ua = u & 0x7fffffffu;
    const int eb = (int)(ua >> 23);
    const int d = min(max(126 - eb, 13), 23);
    const uint32_t r = ((rnd & 0xffffu) << 16) >> (32 - d);
    uint32_t m = (ua + r) & (0xffffffffu << d);
    if (eb < 103) m = (float)(rnd & 0xffffu) < __uint_as_float(ua) * 0x1p40f ? 0x33800000u : 0u;
    const float q = __uint_as_float(m | (u & 0x80000000u));
    return (_Float16)(eb == 255 ? v : q);
}

__device__ __forceinline__ void rd_st_sr(float *p, int64_t i, float v, uint32_t)
{
    __builtin_nontemporal_store(v, p + i);
}
__device__ __forceinline__ void rd_st_sr(bf16_t *p, int64_t i, float v, uint32_t rnd)
{
    p[i].bits = bf16_sr(v, rnd);
}
__device__ __forceinline__ void rd_st_sr(_Float16 *p, int64_t i, float v, uint32_t rnd)
{
    p[i] = f16_sr(v, rnd);
}

// ---- paired access: two x-adjacent slots (index i even) in one 8- or 4-byte access
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void rd_ld2(const float *p, int64_t i, float &a, float &b)
{
    const float2 v = *reinterpret_cast<const float2 *>(p + i);
    a = v.x;
    b = v.y;
}
__device__ __forceinline__ void rd_ld2(const bf16_t *p, int64_t i, float &a, float &b)
{
    const uint32_t u = *reinterpret_cast<const uint32_t *>(p + i);
    a = __uint_as_float(u << 16);
    b = __uint_as_float(u & 0xffff0000u);
}
__device__ __forceinline__ void rd_ld2(const _Float16 *p, int64_t i, float &a, float &b)
{
    const half2_t v = *reinterpret_cast<const half2_t *>(p + i);
    a = (float)v.x;
    b = (float)v.y;
}

// Store a pair; sr selects stochastic rounding with the per-slot random words r0, r1.
__device__ __forceinline__ void rd_st2(float *p, int64_t i, float a, float b, bool, uint32_t,
                                       uint32_t)
{
    *reinterpret_cast<float2 *>(p + i) = make_float2(a, b);
}
__device__ __forceinline__ void rd_st2(bf16_t *p, int64_t i, float a, float b, bool sr, uint32_t r0,
                                       uint32_t r1)
{
    const uint32_t lo = sr ? bf16_sr(a, r0) : bf16_rne(a);
    const uint32_t hi = sr ? bf16_sr(b, r1) : bf16_rne(b);
    *reinterpret_cast<uint32_t *>(p + i) = lo | (hi << 16);
}
__device__ __forceinline__ void rd_st2(_Float16 *p, int64_t i, float a, float b, bool sr,
                                       uint32_t r0, uint32_t r1)
{
    half2_t v;
    v.x = sr ? f16_sr(a, r0) : (_Float16)a;
    v.y = sr ? f16_sr(b, r1) : (_Float16)b;
    *reinterpret_cast<half2_t *>(p + i) = v;
}

// ---- compact layout (B = 8) --------------------------------------------------
// A block stores only its active voxels, in slot order, starting at cbase[b]; the
// plane prefix counts sit in words 14-15 of the block's mask record.
// Number of set bits of the wave-uniform word W in the lanes below this one.
__device__ __forceinline__ uint32_t lanes_below(uint64_t W)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(W >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)W, 0u));
}
// Active slots below plane z of a block (from its mask record).
__device__ __forceinline__ uint32_t plane_prefix(const uint64_t *rec, int z)
{
    return (uint32_t)(rec[14 + (z >> 2)] >> (16 * (z & 3))) & 0xffffu;
}
// Element index of (active) slot `slot` of block b: block-major (cbase NULL) or compact.
__device__ __forceinline__ int64_t slot_index8(const uint32_t *cbase, const uint64_t *mask, int64_t b,
                                               int slot)
{
    if (!cbase) return b * 512 + slot;
    const uint64_t *rec = mask + b * 16;
    const int z = slot >> 6, bit = slot & 63;
    const uint64_t below = bit ? (rec[z] & (~0ull >> (64 - bit))) : 0ull;
    return (int64_t)cbase[b] + plane_prefix(rec, z) + (uint32_t)__popcll(below);
}

// ---- block geometry helpers -------------------------------------------------
template <int B>
struct Blk {
    static constexpr int NS = B * B * B;   // slots per block
    static constexpr int E = B + 2;        // tile edge with halo
    static constexpr int TL = E * E * E;   // tile size (corners unused)
    static constexpr int MW = mask_words(B);
    __device__ static __forceinline__ int tidx(int lx, int ly, int lz)
    {
        return ((lz + 1) * E + (ly + 1)) * E + (lx + 1);
    }
};

// Own active bit of slot s in a mask record.
template <int B>
__device__ __forceinline__ bool own_bit(const uint64_t *rec, int s)
{
    if constexpr (B == 8) return (rec[s >> 6] >> (s & 63)) & 1ull;
    else return (rec[0] >> s) & 1ull;
}

// Face bit `bit` of face f (the neighbour voxel across that face is active).
template <int B>
__device__ __forceinline__ bool face_bit(const uint64_t *rec, int f, int bit)
{
    if constexpr (B == 8) return (rec[8 + f] >> bit) & 1ull;
    else {
        const int w = f < 4 ? 1 : 2;
        const int sh = f < 4 ? 16 * f : 16 * (f - 4);
        return (rec[w] >> (sh + bit)) & 1ull;
    }
}

// Six neighbour activity bits (bit d for direction d in -x,+x,-y,+y,-z,+z order)
// and the wall count (in-box inactive neighbours) of slot (lx,ly,lz) at global
// position (gx,gy,gz) in a box nx*ny*nz.
template <int B>
__device__ __forceinline__ unsigned nb_bits(const uint64_t *rec, int lx, int ly, int lz, int gx,
                                            int gy, int gz, int nx, int ny, int nz, int *nwall)
{
    const int s = (lz * B + ly) * B + lx;
    unsigned m = 0;
    m |= (lx > 0 ? own_bit<B>(rec, s - 1) : face_bit<B>(rec, 0, lz * B + ly)) ? 1u : 0u;
    m |= (lx < B - 1 ? own_bit<B>(rec, s + 1) : face_bit<B>(rec, 1, lz * B + ly)) ? 2u : 0u;
    m |= (ly > 0 ? own_bit<B>(rec, s - B) : face_bit<B>(rec, 2, lz * B + lx)) ? 4u : 0u;
    m |= (ly < B - 1 ? own_bit<B>(rec, s + B) : face_bit<B>(rec, 3, lz * B + lx)) ? 8u : 0u;
    m |= (lz > 0 ? own_bit<B>(rec, s - B * B) : face_bit<B>(rec, 4, ly * B + lx)) ? 16u : 0u;
    m |= (lz < B - 1 ? own_bit<B>(rec, s + B * B) : face_bit<B>(rec, 5, ly * B + lx)) ? 32u : 0u;
    unsigned inbox = 0;
    inbox |= gx > 0 ? 1u : 0u;
    inbox |= gx < nx - 1 ? 2u : 0u;
    inbox |= gy > 0 ? 4u : 0u;
    inbox |= gy < ny - 1 ? 8u : 0u;
    inbox |= gz > 0 ? 16u : 0u;
    inbox |= gz < nz - 1 ? 32u : 0u;
    *nwall = __popc(inbox & ~m);
    return m;
}

// Is a voxel at (gx,gy,gz) on a Dirichlet face plane of a species (dir bits)?
__device__ __forceinline__ bool on_dirichlet(uint32_t dir, int gx, int gy, int gz, int nx, int ny,
                                             int nz)
{
    return ((dir & 1u) && gx == 0) || ((dir & 2u) && gx == nx - 1) ||
           ((dir & 4u) && gy == 0) || ((dir & 8u) && gy == ny - 1) ||
           ((dir & 16u) && gz == 0) || ((dir & 32u) && gz == nz - 1);
}

// The FTCS update of one free voxel of one species (see rd.h):
//   lap = sum over active neighbours q of (c_q - c_p)
//   c'  = c + alpha*lap - (beta + gamma*n_wall)*c + sum_b K_b c_b
// Every caller stages inactive and missing neighbours as exactly 0 (inactive slots
// hold 0 in every field buffer), so the sum over the active neighbours is the sum
// of all six values, and the mirror rule enters through the active count:
//   lap = (((((n_-x + n_+x) + n_-y) + n_+y) + n_-z) + n_+z) - popc(nbm) * c_p
// (one rounding order for every kernel; 6 operations instead of 18).
// The increment  alpha lap - (beta + gamma n_wall) c + sum_b K_b c_b  is formed first and
// added to c once, so c is rounded once per step (forming c + alpha lap and then applying
// each term to it rounded c up to four times).  DTH (FP32 storage with stochastic
// rounding): `dith` (fp32_dither) is added to the increment before that final addition.
// rd_update_n takes the active-neighbour count and the wall count as floats (exact small
// integers), rd_update the neighbour bits; both round identically.
template <int S, bool DTH = false>
__device__ __forceinline__ float rd_update_n(float uc, const float nbv[6], float nact, float nwall,
                                             const SpeciesCoef &k, const float *cen, float dith = 0.0f)
{
    float sum = nbv[0];
#pragma unroll
    for (int d = 1; d < 6; ++d) sum = sum + nbv[d];
    const float lap = fmaf(-nact, uc, sum);
    float inc = k.alpha * lap;
    const float loss = fmaf(k.gamma, nwall, k.beta);
    inc = fmaf(-loss, uc, inc);
#pragma unroll
    for (int b = 0; b < S; ++b) inc = fmaf(k.K[b], cen[b], inc);
    if constexpr (DTH) inc = inc + dith;
    return uc + inc;
}
template <int S, bool DTH = false>
__device__ __forceinline__ float rd_update(float uc, const float nbv[6], unsigned nbm, int nwall,
                                           const SpeciesCoef &k, const float *cen, float dith = 0.0f)
{
    return rd_update_n<S, DTH>(uc, nbv, (float)__popc(nbm & 63u), (float)nwall, k, cen, dith);
}

// Stochastic rounding of FP32 values: a dither (u - 1/2) ulp(c), u in [0, 1) from 16
// random bits, added to the increment makes the round-to-nearest of c + increment + dither
// equal c + increment on average.  Without it, increments below half an ulp of c are lost
// at every step, and a field close to its steady state stops converging about
// (ulp / 2) / (dt * slowest decay rate) away from it.  0 for zero and subnormal c.
__device__ __forceinline__ float fp32_dither(float uc, uint32_t bits16)
{
    // 2^-23 (1 + u) with the 16 bits as the leading mantissa bits, minus 1.5 * 2^-23, is
    // (u - 1/2) 2^-23 exactly; times the power of two of c (c's exponent bits) it is
    // (u - 1/2) ulp(c)
    const float v = __uint_as_float(0x34000000u | (bits16 << 7)) - 0x1.8p-23f;
    return v * __uint_as_float(__float_as_uint(uc) & 0x7f800000u);
}

// Linear index of a voxel in its (nz, ny, nx) box: the key of the stochastic-rounding
// hash, so the random bits do not depend on the block layout.
__device__ __forceinline__ int64_t voxel_id(const GeomInfo &g, int gx, int gy, int gz)
{
    return g.dense0 + ((int64_t)gz * g.ny + gy) * g.nx + gx;
}

// Block position of list entry b.
__device__ __forceinline__ void block_pos(const BlockInfo &bi, int *bx, int *by, int *bz, int *gid)
{
    *bx = bi.xy & 0xffff;
    *by = (bi.xy >> 16) & 0xffff;
    *bz = bi.zg & 0xffff;
    *gid = (bi.zg >> 16) & 0xffff;
}

// Slot of a neighbour block that lies across face f at face coordinates (u, v),
// and the tile index it is staged at.
template <int B>
__device__ __forceinline__ void halo_slot(int f, int u, int v, int *nslot, int *tix)
{
    using K = Blk<B>;
    switch (f) {
    case 0: *nslot = (v * B + u) * B + (B - 1); *tix = ((v + 1) * K::E + (u + 1)) * K::E + 0; break;
    case 1: *nslot = (v * B + u) * B + 0; *tix = ((v + 1) * K::E + (u + 1)) * K::E + (B + 1); break;
    case 2: *nslot = (v * B + (B - 1)) * B + u; *tix = ((v + 1) * K::E + 0) * K::E + (u + 1); break;
    case 3: *nslot = (v * B + 0) * B + u; *tix = ((v + 1) * K::E + (B + 1)) * K::E + (u + 1); break;
    case 4: *nslot = ((B - 1) * B + v) * B + u; *tix = ((0) * K::E + (v + 1)) * K::E + (u + 1); break;
    default: *nslot = (0 * B + v) * B + u; *tix = ((B + 1) * K::E + (v + 1)) * K::E + (u + 1); break;
    }
}

// Generic per-block workgroup shape: B = 8 one block per 256-thread workgroup (two
// voxels per thread); B = 4 four blocks per workgroup, one wave per block.
template <int B>
struct Cfg {
    static constexpr int BPW = B == 8 ? 1 : 4;    // blocks per workgroup
    static constexpr int TPB = 256 / BPW;         // threads per block
    static constexpr int VPT = Blk<B>::NS / TPB;  // voxels per thread
};

// Map a workgroup id to a group of blocks.  With xcd_chunk > 0 the consecutive
// workgroups that the dispatcher sends round-robin to the 8 XCDs are remapped so
// that each XCD walks one contiguous range of the block list (its own L2 then
// holds the +-x / +-y neighbours it needs).
__device__ __forceinline__ int map_group(int wg, int xcd_chunk)
{
    if (xcd_chunk <= 0) return wg;
    return (wg & 7) * xcd_chunk + (wg >> 3);
}

// Stage S fields (species-major, sstride apart) of block b and its six face halos
// into an LDS tile of (B+2)^3 words per field (FP32).  Missing neighbours give 0.
template <typename T, int B>
__device__ __forceinline__ void stage_tile(float (*tile)[Blk<B>::TL], const T *c, int64_t sstride,
                                           int S, int b, const BlockInfo &bi, int lt, bool valid)
{
    using K = Blk<B>;
    using C = Cfg<B>;
    if (!valid) return;
    const int64_t base = (int64_t)b * K::NS;
    for (int s = 0; s < S; ++s) {
#pragma unroll
        for (int k = 0; k < C::VPT; ++k) {
            const int slot = lt + k * C::TPB;
            const int lx = slot % B, ly = (slot / B) % B, lz = slot / (B * B);
            tile[s][K::tidx(lx, ly, lz)] = rd_ld(c, s * sstride + base + slot);
        }
    }
    for (int h = lt; h < 6 * B * B; h += C::TPB) {
        const int f = h / (B * B);
        const int r = h % (B * B);
        int nslot, tix;
        halo_slot<B>(f, r % B, r / B, &nslot, &tix);
        const int n = bi.nbr[f];
        for (int s = 0; s < S; ++s)
            tile[s][tix] = n >= 0 ? rd_ld(c, s * sstride + (int64_t)n * K::NS + nslot) : 0.0f;
    }
}

// Wave-level FP64 sum in a fixed butterfly order (deterministic).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
