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

__device__ __forceinline__ void rd_st(float *p, int64_t i, float v) { p[i] = v; }
__device__ __forceinline__ void rd_st(bf16_t *p, int64_t i, float v)
{
    // round to nearest even on the upper 16 bits; NaN stays NaN (quiet bit set)
    uint32_t u = __float_as_uint(v);
    uint16_t r;
    if ((u & 0x7fffffffu) > 0x7f800000u) {
        r = (uint16_t)((u >> 16) | 0x40u);
    } else {
        u += 0x7fffu + ((u >> 16) & 1u);
        r = (uint16_t)(u >> 16);
    }
    p[i].bits = r;
}
__device__ __forceinline__ void rd_st(_Float16 *p, int64_t i, float v) { p[i] = (_Float16)v; }

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

__device__ __forceinline__ uint32_t sr_bits(int64_t slot, int species, uint32_t step, uint32_t seed)
{
    uint32_t k = mix32(step * 4u + (uint32_t)species + seed * 0x9e3779b9u);
    return mix32((uint32_t)slot ^ mix32((uint32_t)(slot >> 32) ^ k));
}

// Store with stochastic rounding: round up with probability equal to the distance
// from the lower neighbour, in units of the storage spacing (unbiased on average).
__device__ __forceinline__ void rd_st_sr(float *p, int64_t i, float v, uint32_t) { p[i] = v; }
__device__ __forceinline__ void rd_st_sr(bf16_t *p, int64_t i, float v, uint32_t rnd)
{
    // BF16 is the upper half of the FP32 pattern: adding 16 random bits below the cut
    // and truncating rounds the magnitude up with probability (low bits) / 2^16
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7f800000u) == 0x7f800000u) {  // inf / NaN: nearest
        rd_st(p, i, v);
        return;
    }
    u += rnd & 0xffffu;
    p[i].bits = (uint16_t)(u >> 16);
}
__device__ __forceinline__ void rd_st_sr(_Float16 *p, int64_t i, float v, uint32_t rnd)
{
    const _Float16 h = (_Float16)v;
    const float hf = (float)h;
    if (hf == v || !isfinite(v) || !isfinite(hf)) {
        p[i] = h;
        return;
    }
    // the FP16 neighbour of h on the other side of v
    uint16_t b = __builtin_bit_cast(uint16_t, h);
    const bool neg = (b & 0x8000u) != 0;
    const bool mag = (b & 0x7fffu) != 0;
    uint16_t ob;
    if (v > hf) ob = neg ? (mag ? (uint16_t)(b - 1) : (uint16_t)0x0001u) : (uint16_t)(b + 1);
    else ob = neg ? (uint16_t)(b + 1) : (mag ? (uint16_t)(b - 1) : (uint16_t)0x8001u);
    const _Float16 o = __builtin_bit_cast(_Float16, ob);
    const float of = (float)o;
    const float lo = fminf(hf, of), hi = fmaxf(hf, of);
    const float prob_up = (v - lo) / (hi - lo);
    const float u01 = (float)(rnd >> 8) * (1.0f / 16777216.0f);
    p[i] = u01 < prob_up ? (hf > of ? h : o) : (hf > of ? o : h);
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
//   lap = sum over active neighbours, in order -x,+x,-y,+y,-z,+z, of (c_q - c_p)
//   c'  = c + alpha*lap - (beta + gamma*n_wall)*c + sum_b K_b c_b
__device__ __forceinline__ float rd_update(float uc, const float nbv[6], unsigned nbm, int nwall,
                                           const SpeciesCoef &k, const float *cen, int S)
{
    float lap = 0.0f;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        const float t = nbv[d] - uc;
        lap = ((nbm >> d) & 1u) ? lap + t : lap;
    }
    float r = fmaf(k.alpha, lap, uc);
    const float loss = fmaf(k.gamma, (float)nwall, k.beta);
    r = fmaf(-loss, uc, r);
    for (int b = 0; b < S; ++b) r = fmaf(k.K[b], cen[b], r);
    return r;
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

// Wave-level FP64 sum in a fixed butterfly order (deterministic).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
