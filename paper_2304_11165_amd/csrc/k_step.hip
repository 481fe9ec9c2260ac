// k_step.hip -- the sparse-block FTCS step, its FP64 reductions and the dense <->
// block-major layout kernels, for gfx950 (wave64, 160 KB LDS per CU).
//
// Step kernel (paper: FTCS with the mirror rule applied inside the stencil,
// sections "Discretization and numerical methods" and "Parallel implementation"):
//   * B = 8: k_step8z, one wave per block with each lane walking a z-column (the
//     fastest); k_step8, one 256-thread workgroup per block, two voxels per thread;
//     k_step8p, a persistent prefetching grid.  B = 4: k_step4w, one wave per block,
//     four blocks per workgroup, one voxel per thread.
//   * The block and its face halos (read through the neighbour list) are staged as
//     FP32 in LDS tiles; inactive and missing neighbours are staged as exact zeros.
//   * Activity of the six neighbours comes from the block's mask record (own bits
//     plus the neighbours' face bits), so no neighbour mask is read.
//   * Inactive slots are 0 in every field buffer (zero-filled on upload).  The
//     default kernels predicate every load on the activity of the voxel it reads and
//     store whole sectors that hold an active voxel (sector_active), so sectors
//     without active voxels are never moved;
//     the persistent kernel stores 0 into inactive slots.  Dirichlet voxels are
//     copied through.
// The stencil is HBM-bound (about 2 FLOP per byte), so there is no MFMA here.
#include <hip/hip_cooperative_groups.h>

#include "rd_device.h"

namespace {

// Stochastic rounding key of this launch (wave-uniform; 0 when rounding to nearest).
__device__ __forceinline__ uint32_t launch_key(const StepArgs &a)
{
    return a.sround ? sr_key(*a.ctr + a.ctr_off, a.seed) : 0u;
}
// Random word of one voxel (only used with stochastic rounding).
__device__ __forceinline__ uint32_t voxel_bits(const StepArgs &a, uint32_t key, const GeomInfo &g, int gx, int gy,
                                               int gz)
{
    return a.sround ? sr_voxel(g, gx, gy, gz, key) : 0u;
}

// Store one updated value of species s (round to nearest, or stochastic rounding
// with the voxel's random word h when enabled).  PLAIN: an ordinary store also for FP32
// (the compact layout's plane runs share 128-byte lines with their neighbours, which a
// nontemporal store would send to memory half written).
template <typename T, bool PLAIN = false>
__device__ __forceinline__ void store_val(const StepArgs &a, T *cout, int s, int64_t idx, uint32_t h,
                                          float r)
{
    if constexpr (PLAIN && sizeof(T) == 4) cout[idx] = r;
    else if (a.sround) rd_st_sr(cout, idx, r, sr_species(h, s));
    else rd_st(cout, idx, r);
}
// p advanced by a 32-bit byte offset: a wave-uniform base plus a zero-extended 32-bit
// offset, the form of a global access with a scalar base and a 32-bit vector offset (no
// 64-bit address arithmetic per access).  The offsets fit: a compact species buffer holds
// fewer than 2^30 values, and block-layout offsets stay inside one block's slab.
template <typename T>
__device__ __forceinline__ T *at_byte(T *p, uint32_t off)
{
    return (T *)((char *)p + (uint64_t)off);
}
template <typename T>
__device__ __forceinline__ const T *at_byte(const T *p, uint32_t off)
{
    return (const T *)((const char *)p + (uint64_t)off);
}
// A wave-uniform pointer pinned to scalar registers, so that the compiler keeps it as the
// scalar base of the accesses above instead of folding it into each 64-bit vector address.
// (The field buffers are device memory: the pointer is rebuilt in the global address
// space, so the accesses stay global ones.)
template <typename T>
__device__ __forceinline__ T *uniform_ptr(T *p)
{
    typedef __attribute__((address_space(1))) T GT;
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (T *)(GT *)(((uint64_t)hi << 32) | lo);
}

// The same with the rounding mode fixed at compile time (SR: stochastic rounding on).
template <typename T, bool PLAIN, bool SR>
__device__ __forceinline__ void store_val_ct(T *cout, int s, int64_t idx, uint32_t h, float r)
{
    if constexpr (PLAIN && sizeof(T) == 4) cout[idx] = r;
    else if constexpr (SR) rd_st_sr(cout, idx, r, sr_species(h, s));
    else rd_st(cout, idx, r);
}

// Branch-free update of voxel (lx, ly, lz) of a B = 8 block, all species.  W, Wm, Wp
// are the active-bit words of planes lz, lz-1, lz+1 (or the -z / +z face words at the
// block edge); fx0..fy1 the +-x / +-y face words.  ts points at the voxel's centre
// word in the species-0 tile, sstr is the word distance between species tiles and
// (oy, oz) the y / z neighbour offsets of the tile layout.  onf: bit d set when the
// voxel lies on box face d, which marks both Dirichlet planes (onf & dir) and
// out-of-box neighbours (no wall there).
template <int S, bool DTH>
__device__ __forceinline__ void vox8(const StepArgs &a, const float *ts, int sstr, int oy, int oz,
                                     uint64_t W, uint64_t Wm, uint64_t Wp, uint64_t fx0,
                                     uint64_t fx1, uint64_t fy0, uint64_t fy1, int lx, int ly,
                                     int lz, unsigned onf, const float *cen, float *out, uint32_t hd)
{
    const int bit = ly * 8 + lx;
    const uint64_t fxb = (uint64_t)1 << (lz * 8 + ly), fyb = (uint64_t)1 << (lz * 8 + lx);
    const uint64_t ob = (uint64_t)1 << bit;
    unsigned m = 0;
    m |= ((lx > 0 ? (W & (ob >> 1)) : (fx0 & fxb)) != 0) ? 1u : 0u;
    m |= ((lx < 7 ? (W & (ob << 1)) : (fx1 & fxb)) != 0) ? 2u : 0u;
    m |= ((ly > 0 ? (W & (ob >> 8)) : (fy0 & fyb)) != 0) ? 4u : 0u;
    m |= ((ly < 7 ? (W & (ob << 8)) : (fy1 & fyb)) != 0) ? 8u : 0u;
    m |= (Wm & ob) != 0 ? 16u : 0u;
    m |= (Wp & ob) != 0 ? 32u : 0u;
    const bool act = (W & ob) != 0;
    const int nwall = __popc(~onf & ~m & 0x3fu);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const float *p = ts + s * sstr;
        const float nbv[6] = {p[-1], p[1], p[-oy], p[oy], p[-oz], p[oz]};
        const float dth = DTH ? fp32_dither(cen[s], sr_species(hd, s)) : 0.0f;
        const float upd = rd_update<S, DTH>(cen[s], nbv, m, nwall, a.coef[s], cen, dth);
        const bool isd = (onf & a.coef[s].dir) != 0u;
        out[s] = act ? (isd ? cen[s] : upd) : 0.0f;
    }
}

__device__ __forceinline__ unsigned box_faces(const GeomInfo &g, int gx, int gy, int gz)
{
    return (gx == 0 ? 1u : 0u) | (gx == g.nx - 1 ? 2u : 0u) | (gy == 0 ? 4u : 0u) |
           (gy == g.ny - 1 ? 8u : 0u) | (gz == 0 ? 16u : 0u) | (gz == g.nz - 1 ? 32u : 0u);
}

// Update of one voxel from its precomputed neighbour code (bits 0-5 active neighbours,
// bit 6 active) and its box-face bits onf (0 for blocks away from the box boundary).
// Same arithmetic as every other variant (rd_update).
template <int S, bool DTH>
__device__ __forceinline__ void vox_code(const StepArgs &a, const float *ts, int sstr, int oy,
                                         int oz, unsigned code, unsigned onf, const float *cen,
                                         float *out, uint32_t hd)
{
    const unsigned m = code & 63u;
    const bool act = (code & 64u) != 0u;
    const int nwall = __popc(~onf & ~m & 0x3fu);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const float *p = ts + s * sstr;
        const float nbv[6] = {p[-1], p[1], p[-oy], p[oy], p[-oz], p[oz]};
        const float dth = DTH ? fp32_dither(cen[s], sr_species(hd, s)) : 0.0f;
        const float upd = rd_update<S, DTH>(cen[s], nbv, m, nwall, a.coef[s], cen, dth);
        const bool isd = (onf & a.coef[s].dir) != 0u;
        out[s] = act ? (isd ? cen[s] : upd) : 0.0f;
    }
}

// Does a B = 8 block at (bx, by, bz) touch the box boundary (uniform per block)?
__device__ __forceinline__ bool boundary_block(const GeomInfo &g, int bx, int by, int bz)
{
    return bx == 0 || by == 0 || bz == 0 || bx * 8 + 8 >= g.nx || by * 8 + 8 >= g.ny ||
           bz * 8 + 8 >= g.nz;
}

// B = 4 step: one wave per block (lane = slot), four independent blocks per
// workgroup.  Each wave stages its block and the 6 x 16 halo values in a private
// LDS tile of 6^3 words per species, then updates its 64 voxels from the neighbour
// codes.  Only wave-level ordering is needed (no workgroup barrier).
// DTH (FP32 storage with stochastic rounding): the update takes a dither (fp32_dither).
template <typename T, int S, bool DTH>
__global__ __launch_bounds__(256) void k_step4w(StepArgs a)
{
    constexpr int E = 6, E2 = 36, TLW = 216;
    __shared__ float tile[4][S][TLW];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int grp = map_group(blockIdx.x, a.xcd_chunk);
    const int b = __builtin_amdgcn_readfirstlane(grp * 4 + wv);
    if (b >= a.nb) return;  // the whole wave leaves; no workgroup barrier below
    const T *cin = (const T *)a.cin;
    T *cout = (T *)a.cout;
    const int64_t base = (int64_t)b * 64;
    const int lx = lane & 3, ly = (lane >> 2) & 3, lz = lane >> 4;

    // Wave-uniform mask record: own word, faces 0-3 (16 bits each) and faces 4-5.
    // Lane l's bit is l in all three (slot l; face l / 16 at (u, v) with bit
    // v * 4 + u = l % 16), so every load is predicated on the voxel it reads.
    const uint64_t *rec = a.mask + (int64_t)b * 3;
    const uint64_t Wo = rec[0], Wf0 = rec[1], Wf1 = rec[2];
    const bool act = (Wo >> lane) & 1ull;
    const bool two = lane < 32;
    const bool e0 = (Wf0 >> lane) & 1ull, e1 = two && ((Wf1 >> lane) & 1ull);

    // halo: lanes 16f..16f+15 fetch face f (f = 0..3); lanes 0..31 also faces 4, 5.
    // The six neighbour indices are loaded once as wave-uniform values and each lane
    // selects its face's by value (a select between memory reads of nbr[f] was once
    // lowered to divergent control flow that gave the +y lanes the -y index).  A face
    // bit is set only when the neighbour block exists; the address still falls back
    // to the block itself so that it is valid in every lane.
    const int f0 = lane >> 4, f1 = 4 + (lane >> 4);
    const BlockInfo bi0 = a.info[b];
    int n0 = bi0.nbr[0];
    n0 = f0 == 1 ? bi0.nbr[1] : n0;
    n0 = f0 == 2 ? bi0.nbr[2] : n0;
    n0 = f0 == 3 ? bi0.nbr[3] : n0;
    const int n1 = (f1 & 1) ? bi0.nbr[5] : bi0.nbr[4];  // lanes 32..63 never load (e1 = 0)
    typedef typename RawOf<T>::type R;
    R rc[S], rh0[S], rh1[S];
#pragma unroll
    for (int s = 0; s < S; ++s) rc[s] = ld_raw(cin, s * a.sstride + base + lane, act);
    const unsigned code = act ? (unsigned)a.code[base + lane] : 0u;
    const int u = lane & 3, v = (lane >> 2) & 3;
    int ns0, tx0, ns1 = 0, tx1 = 0;
    halo_slot<4>(f0, u, v, &ns0, &tx0);
    halo_slot<4>(f1 & 5, u, v, &ns1, &tx1);
    const int64_t hb0 = (int64_t)(n0 >= 0 ? n0 : b) * 64 + ns0;
#pragma unroll
    for (int s = 0; s < S; ++s) rh0[s] = ld_raw(cin, s * a.sstride + hb0, e0);
    const int64_t hb1 = (int64_t)(n1 >= 0 ? n1 : b) * 64 + ns1;
#pragma unroll
    for (int s = 0; s < S; ++s) rh1[s] = ld_raw(cin, s * a.sstride + hb1, e1);
    // all loads are issued; convert to FP32
    float c[S];
    const int t = ((lz + 1) * E + (ly + 1)) * E + (lx + 1);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        c[s] = from_raw<T>(rc[s]);
        tile[wv][s][t] = c[s];
        tile[wv][s][tx0] = from_raw<T>(rh0[s]);
        if (two) tile[wv][s][tx1] = from_raw<T>(rh1[s]);
    }
    // the wave's LDS writes complete before its reads of other lanes' words
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    const BlockInfo bi = a.info[b];
    int bx, by, bz, gid;
    block_pos(bi, &bx, &by, &bz, &gid);
    const GeomInfo g = a.geom[gid];
    const int gx = bx * 4 + lx, gy = by * 4 + ly, gz = bz * 4 + lz;
    const bool bnd = bx == 0 || by == 0 || bz == 0 || bx * 4 + 4 >= g.nx || by * 4 + 4 >= g.ny ||
                     bz * 4 + 4 >= g.nz;
    unsigned onf = 0u;
    if (bnd) onf = box_faces(g, gx, gy, gz);
    float res[S];
    const uint32_t h = voxel_bits(a, launch_key(a), g, gx, gy, gz);
    vox_code<S, DTH>(a, &tile[wv][0][t], TLW, E, E2, code, onf, c, res, h);
    // whole sectors only; an inactive slot of an active sector stores its 0 again
    if (sector_active<T>(Wo, lane)) {
#pragma unroll
        for (int s = 0; s < S; ++s) store_val(a, cout, s, s * a.sstride + base + lane, h, res[s]);
    }
}

// B = 8 step.  Wave w (0..3) owns the planes lz = w and lz = w + 4 of the block, lane
// (lx, ly) = (l % 8, l / 8), so every mask word a wave needs (own planes lz-1..lz+1
// and the six face words) is wave-uniform and read with scalar loads.  Each thread
// issues all of its global loads (2 own values and 1-2 halo values per species)
// before the first wait; the halo of face w (x / y faces) and of face 4 + w (z faces,
// waves 0-1) goes through the wave-uniform neighbour index.
template <typename T, int S, bool DTH>
__global__ __launch_bounds__(256) void k_step8(StepArgs a)
{
    using K = Blk<8>;
    __shared__ float tile[S][K::TL];
    const int b = map_group(blockIdx.x, a.xcd_chunk);
    if (b >= a.nb) return;  // the whole workgroup leaves together
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int lx = lane & 7, ly = lane >> 3;
    const T *cin = (const T *)a.cin;
    T *cout = (T *)a.cout;
    const int64_t base = (int64_t)b * K::NS;
    const int32_t *nbr = a.info[b].nbr;
    // Wave-uniform mask words: own planes w and w + 4, face w and (waves 0-1) face
    // 4 + w.  Lane l's bit is l in each of them (own slot (lx, ly); face coordinates
    // (u, v) = (lx, ly) with bit v * 8 + u), so every load below is predicated on
    // the activity of the voxel it reads: only sectors holding active voxels move.
    const uint64_t *rec = a.mask + (int64_t)b * K::MW;
    const bool zf = w < 2;
    const uint64_t Wo0 = rec[w], Wo1 = rec[w + 4], Wf0 = rec[8 + w];
    const uint64_t Wf1 = zf ? rec[12 + w] : 0ull;
    const bool a0 = (Wo0 >> lane) & 1ull, a1 = (Wo1 >> lane) & 1ull;
    const bool e0 = (Wf0 >> lane) & 1ull, e1 = (Wf1 >> lane) & 1ull;

    typedef typename RawOf<T>::type R;
    R r0[S], r1[S], rh0[S], rh1[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        r0[s] = ld_raw(cin, s * a.sstride + base + w * 64 + lane, a0);
        r1[s] = ld_raw(cin, s * a.sstride + base + (w + 4) * 64 + lane, a1);
    }
    const unsigned cd0 = a0 ? (unsigned)a.code[base + w * 64 + lane] : 0u;
    const unsigned cd1 = a1 ? (unsigned)a.code[base + (w + 4) * 64 + lane] : 0u;
    // halos: a face bit is set only when the neighbour block exists; the address
    // still falls back to the block itself so that it is valid in every lane
    int ns0, tx0, ns1 = 0, tx1 = 0;
    halo_slot<8>(w, lx, ly, &ns0, &tx0);
    const int n0 = nbr[w];
    const int64_t hb0 = (int64_t)(n0 >= 0 ? n0 : b) * K::NS + ns0;
#pragma unroll
    for (int s = 0; s < S; ++s) rh0[s] = ld_raw(cin, s * a.sstride + hb0, e0);
    halo_slot<8>(4 + (w & 1), lx, ly, &ns1, &tx1);  // waves 2-3 have no z face
    const int n1 = nbr[4 + (w & 1)];
    const int64_t hb1 = (int64_t)(n1 >= 0 ? n1 : b) * K::NS + ns1;
#pragma unroll
    for (int s = 0; s < S; ++s) rh1[s] = ld_raw(cin, s * a.sstride + hb1, e1);  // e1 = 0 there
    // all loads are issued; convert to FP32
    float c0[S], c1[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        c0[s] = from_raw<T>(r0[s]);
        c1[s] = from_raw<T>(r1[s]);
        tile[s][K::tidx(lx, ly, w)] = c0[s];
        tile[s][K::tidx(lx, ly, w + 4)] = c1[s];
        tile[s][tx0] = from_raw<T>(rh0[s]);
        if (zf) tile[s][tx1] = from_raw<T>(rh1[s]);
    }
    __syncthreads();

    const BlockInfo bi = a.info[b];
    int bx, by, bz, gid;
    block_pos(bi, &bx, &by, &bz, &gid);
    const GeomInfo g = a.geom[gid];
    const int gx = bx * 8 + lx, gy = by * 8 + ly;
    const bool bnd = boundary_block(g, bx, by, bz);
    const uint32_t key = launch_key(a);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int lz = w + 4 * k;
        const int gz = bz * 8 + lz;
        const int slot = lz * 64 + lane;
        unsigned onf = 0u;
        if (bnd) onf = box_faces(g, gx, gy, gz);
        float cen[S], res[S];
#pragma unroll
        for (int s = 0; s < S; ++s) cen[s] = k == 0 ? c0[s] : c1[s];
        const uint32_t h = voxel_bits(a, key, g, gx, gy, gz);
        vox_code<S, DTH>(a, &tile[0][K::tidx(lx, ly, lz)], K::TL, K::E, K::E * K::E, k == 0 ? cd0 : cd1,
                         onf, cen, res, h);
        // whole sectors only; an inactive slot of an active sector stores its 0 again
        if (sector_active<T>(k == 0 ? Wo0 : Wo1, lane)) {
#pragma unroll
            for (int s = 0; s < S; ++s) store_val(a, cout, s, s * a.sstride + base + slot, h, res[s]);
        }
    }
}

// B = 8 step, one wave per block and four blocks per workgroup.  Lane l = (lx, ly)
// walks its z-column lz = 0..7: the -z / +z neighbours of a voxel are the values
// above and below it in the lane's own registers (the -z / +z face halos at the
// column ends), and only the +-x / +-y neighbours go through LDS, one plane at a
// time: a wave-private 10 x 10 tile per species holds plane lz and its ring of side
// halos (800 bytes per wave for two species, so LDS does not limit residency).
// Every global load of the block is issued before the first plane is computed, and
// every per-block cost (mask words, neighbour list, addresses, predicates) is paid
// once per 8 voxels of a lane.
// The four blocks of a workgroup are consecutive list entries, and an existing +x
// neighbour of entry b is always entry b + 1 (ascending linear ids, x fastest).  So
// With XCH, x-adjacent blocks of one workgroup hand each other their x = 0 / x = 7
// planes through LDS (one workgroup barrier) instead of re-reading the neighbour's
// strided column from L2: an x face touches every 128-byte line of the neighbour
// block.  It pays with FP32 storage; the barrier costs more than it saves for the
// latency-bound 16-bit forms, so both are autotuner candidates.
// Active-neighbour counts of a B = 8 block, one 32-bit word per lane (x, y) of the
// column kernel: bits 3z..3z+2 hold the count of voxel (x, y, z) (0..6), equal to the
// popcount of its code's six neighbour bits.  Built once per geometry from the mask
// records: for each plane and direction a 64-bit word holds at bit l whether lane l's
// neighbour in that direction is active (shifts of the plane word inside the block, the
// neighbours' face words across its faces); three full adders sum the six words
// bit-sliced, and lane l's count is bit l of the three sums.
__device__ __forceinline__ uint64_t transpose8x8(uint64_t x)
{
    // bit r*8+c -> bit c*8+r: delta swaps of 1x1, 2x2 and 4x4 sub-blocks
    uint64_t t = (x ^ (x >> 7)) & 0x00AA00AA00AA00AAull;
    x = x ^ t ^ (t << 7);
    t = (x ^ (x >> 14)) & 0x0000CCCC0000CCCCull;
    x = x ^ t ^ (t << 14);
    t = (x ^ (x >> 28)) & 0x00000000F0F0F0F0ull;
    x = x ^ t ^ (t << 28);
    return x;
}
__device__ __forceinline__ void full_add64(uint64_t a, uint64_t b, uint64_t c, uint64_t &sum, uint64_t &carry)
{
    const uint64_t t = a ^ b;
    sum = t ^ c;
    carry = (a & b) | (c & t);
}

// One thread per (block, lane): the lane's count word.
__global__ void k_count_words8(const uint64_t *__restrict__ mask, uint32_t *__restrict__ ncnt, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t *rec = mask + (i >> 6) * 16;
    const int l = (int)(i & 63);
    constexpr uint64_t COL0 = 0x0101010101010101ull;  // lanes with x = 0
    // face words: -x, +x, -y, +y, -z, +z at 8..13, face coordinates (u, v), bit v*8+u;
    // the x faces' (u, v) = (y, z), so their transpose holds column x = 0 of plane z at
    // bits y*8
    const uint64_t tx0 = transpose8x8(rec[8]), tx1 = transpose8x8(rec[9]);
    uint32_t w = 0u;
    for (int z = 0; z < 8; ++z) {
        const uint64_t P = rec[z];
        const uint64_t xm = ((P << 1) & ~COL0) | ((tx0 >> z) & COL0);
        const uint64_t xp = ((P >> 1) & ~(COL0 << 7)) | (((tx1 >> z) & COL0) << 7);
        const uint64_t ym = (P << 8) | ((rec[10] >> (8 * z)) & 0xffull);
        const uint64_t yp = (P >> 8) | (((rec[11] >> (8 * z)) & 0xffull) << 56);
        const uint64_t zm = z > 0 ? rec[z - 1] : rec[12];
        const uint64_t zp = z < 7 ? rec[z + 1] : rec[13];
        uint64_t s1, c1, s2, c2, n1, n2;
        full_add64(xm, xp, ym, s1, c1);
        full_add64(yp, zm, zp, s2, c2);
        full_add64(c1, c2, s1 & s2, n1, n2);
        const uint32_t cnt = (uint32_t)(((s1 ^ s2) >> l) & 1ull) + 2u * (uint32_t)((n1 >> l) & 1ull) +
                             4u * (uint32_t)((n2 >> l) & 1ull);
        w |= cnt << (3 * z);
    }
    ncnt[i] = w;
}

namespace z8 {
__device__ __forceinline__ int pix(int x, int y) { return (y + 1) * 10 + (x + 1); }
}  // namespace z8

// With CMP the fields and neighbour codes hold only the active voxels (compact
// layout): plane z of block b starts at cbase[b] + (active slots below plane z) and a
// lane's voxel sits at the number of active lanes below it; a side halo value is found
// from the neighbour's plane word and prefix count (one record line), a z halo from
// the face word.  Loads, arithmetic and stored values are those of the block-major
// layout, so both give the same bits; stores cover the active voxels only.
// DTH: stochastic rounding (FP32: the dither added to each increment; 16-bit: the
// rounding of the stores).
// One workgroup's work: the four blocks of group grp (list entries 4 grp .. 4 grp + 3).
template <typename T, int S, bool XCH, bool CMP, bool DTH>
__device__ __forceinline__ void step8z_group(const StepArgs &a, int grp)
{
    __shared__ float tile[4][S][100];
    __shared__ float xch[4][2][S][64];  // x = 0 / x = 7 planes of each wave's block, [z * 8 + y]
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int b = __builtin_amdgcn_readfirstlane(grp * 4 + wv);
    if (b >= a.nb) {  // past the end of the list (with XCH: after the one barrier)
        if (XCH) __syncthreads();
        return;
    }
    const T *cin = (const T *)a.cin;
    T *cout = (T *)a.cout;
    // per-species bases in scalar registers: the species buffer (CMP) or the block's slab
    // in it; every access below is a base plus a 32-bit byte offset
    const T *cinb[S];
    T *coutb[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int64_t o = s * a.sstride + (CMP ? 0 : (int64_t)b * 512);
        cinb[s] = uniform_ptr(cin + o);
        coutb[s] = uniform_ptr(cout + o);
    }
    const int lx = lane & 7, ly = lane >> 3;
    // the block record whole and unconditionally: one scalar load, issued with the mask
    // record's, instead of a load per neighbour index behind the tests below
    const BlockInfo bi = a.info[b];
    const int32_t *nbr = bi.nbr;
    // x neighbours inside this workgroup (wave-uniform; only with XCH)
    const bool xm_in = XCH && wv > 0 && nbr[0] == b - 1;
    const bool xp_in = XCH && wv < 3 && nbr[1] == b + 1;
    // CMP: what the side-halo positions are made of, loaded first so that their latency
    // passes under the mask-record and plane loads: the block's halo record (ends / starts
    // of the y neighbours' plane v = ly, the z neighbours' run bounds) and, for the x
    // neighbours (list entries b - 1 and b + 1, clamped to the list; read only where the
    // neighbour exists), plane v's word and start position
    uint32_t hym = 0u, hyp = 0u, hzm = 0u, hzp = 0u, xmb = 0u, xpb = 0u;
    uint64_t xmw = 0ull, xpw = 0ull;
    if constexpr (CMP) {
        const uint32_t *hr = a.hrec + (int64_t)b * 32;
        hym = hr[ly];
        hyp = hr[8 + ly];
        hzm = hr[16];
        hzp = hr[17];
        const int bm = b > 0 ? b - 1 : b, bp = b + 1 < a.nb ? b + 1 : b;
        const uint64_t *rm = a.mask + (int64_t)bm * 16, *rp = a.mask + (int64_t)bp * 16;
        xmw = rm[ly];
        xpw = rp[ly];
        xmb = a.cbase[bm] + plane_prefix(rm, ly);
        xpb = a.cbase[bp] + plane_prefix(rp, ly);
    }
    // mask record: own plane words 0-7, face words 8-13; lane l's bit is l in each
    // (own slot (lx, ly) of a plane; face coordinates (u, v) = (lx, ly), bit v*8+u)
    const uint64_t *rec = a.mask + (int64_t)b * 16;
    uint64_t Wo[8], Wf[6];
#pragma unroll
    for (int z = 0; z < 8; ++z) Wo[z] = rec[z];
#pragma unroll
    for (int f = 0; f < 6; ++f) Wf[f] = rec[8 + f];

    // element index of the lane's voxel in plane z (valid where the voxel is active)
    uint32_t oi[8];  // from the species base (CMP) or the block's slab
    if constexpr (CMP) {
        uint32_t acc = a.cbase[b];
#pragma unroll
        for (int z = 0; z < 8; ++z) {
            oi[z] = acc + lanes_below(Wo[z]);
            acc += (uint32_t)__popcll(Wo[z]);
        }
    } else {
#pragma unroll
        for (int z = 0; z < 8; ++z) oi[z] = (uint32_t)(z * 64 + lane);
    }

    typedef typename RawOf<T>::type R;
    R rc[S][8], rh[6][S];
    // the lane's active-neighbour counts of its 8 voxels (3 bits each)
    const uint32_t ncw = a.ncnt[(int64_t)b * 64 + lane];
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        // the plane's loads under one predicate (0 where the voxel is inactive)
#pragma unroll
        for (int s = 0; s < S; ++s) rc[s][z] = (R)0;
        if (lane_bit(Wo[z])) {
#pragma unroll
            for (int s = 0; s < S; ++s) rc[s][z] = ld_raw(at_byte(cinb[s], oi[z] * (uint32_t)sizeof(T)), 0);
        }
    }
    // face halos, one value per lane and face: lane (u, v) = (lx, ly) reads the
    // neighbour slot across face f at face coordinates (u, v); a face bit is set only
    // when the neighbour block exists, the address falls back to the block itself
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        int ns;
        switch (f) {
        case 0: ns = (ly * 8 + lx) * 8 + 7; break;  // (x=7, y=u, z=v)
        case 1: ns = (ly * 8 + lx) * 8 + 0; break;  // (x=0, y=u, z=v)
        case 2: ns = (ly * 8 + 7) * 8 + lx; break;  // (x=u, y=7, z=v)
        case 3: ns = (ly * 8 + 0) * 8 + lx; break;  // (x=u, y=0, z=v)
        case 4: ns = (7 * 8 + ly) * 8 + lx; break;  // (x=u, y=v, z=7)
        default: ns = (0 * 8 + ly) * 8 + lx; break; // (x=u, y=v, z=0)
        }
        const int n = nbr[f];
        const int nn = n >= 0 ? n : b;
        const uint64_t need = (f == 0 && xm_in) || (f == 1 && xp_in) ? 0ull : Wf[f];
#pragma unroll
        for (int s = 0; s < S; ++s) rh[f][s] = (R)0;
        int64_t hb;
        if constexpr (CMP) {
            // every position follows from b alone (no load waits for the neighbour
            // table), from the values loaded at the top
            if (f == 4) {  // plane 7 of the -z neighbour: its last popc(Wf[4]) voxels
                hb = (int64_t)hzm - __popcll(Wf[4]) + lanes_below(Wf[4]);
            } else if (f == 5) {  // plane 0 of the +z neighbour
                hb = (int64_t)hzp + lanes_below(Wf[5]);
            } else if (f < 2) {  // slot (x = 7 / 0, y = u = lx) of plane v = ly: the plane's
                                 // start plus its active slots below that one
                const int bit = lx * 8 + (f == 0 ? 7 : 0);
                const uint64_t below = ((f == 0 ? xmw : xpw) & ((1ull << bit) - 1ull));
                hb = (int64_t)(f == 0 ? xmb : xpb) + __popcll(below);
            } else {  // row y = 7 / y = 0 of plane v = ly at x = u = lx: the end / start of
                      // that plane less / plus the row's active voxels at or after / before u
                const uint32_t row = (uint32_t)(Wf[f] >> (8 * ly)) & 0xffu;
                if (f == 2) hb = (int64_t)hym - __popc(row >> lx);
                else hb = (int64_t)hyp + __popc(row & ((1u << lx) - 1u));
            }
        } else {
            hb = ns;  // in the neighbour's slab
        }
        if (lane_bit(need)) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const T *hbase = CMP ? cinb[s] : uniform_ptr(cin + s * a.sstride + (int64_t)nn * 512);
                rh[f][s] = ld_raw(at_byte(hbase, (uint32_t)hb * (uint32_t)sizeof(T)), 0);
            }
        }
    }
    // all loads are issued; convert to FP32
    float c[S][8], side[4][S], zlo[S], zhi[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
#pragma unroll
        for (int z = 0; z < 8; ++z) c[s][z] = from_raw<T>(rc[s][z]);
#pragma unroll
        for (int f = 0; f < 4; ++f) side[f][s] = from_raw<T>(rh[f][s]);
        zlo[s] = from_raw<T>(rh[4][s]);
        zhi[s] = from_raw<T>(rh[5][s]);
    }
    // hand the x = 0 / x = 7 planes to the x neighbours of this workgroup; inactive
    // slots are 0 already, as a predicated halo load would give
    if (XCH) {
        if (lx == 0 || lx == 7) {
#pragma unroll
            for (int s = 0; s < S; ++s)
#pragma unroll
                for (int z = 0; z < 8; ++z) xch[wv][lx == 7 ? 1 : 0][s][z * 8 + ly] = c[s][z];
        }
        __syncthreads();
        // face coordinates (u, v) = (lx, ly) of an x face are (y, z)
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (xm_in) side[0][s] = xch[wv - 1][1][s][ly * 8 + lx];
            if (xp_in) side[1][s] = xch[wv + 1][0][s][ly * 8 + lx];
        }
    }

    int bx, by, bz, gid;
    block_pos(bi, &bx, &by, &bz, &gid);
    const GeomInfo g = a.geom[gid];
    const int gx = bx * 8 + lx, gy = by * 8 + ly;
    const bool bnd = boundary_block(g, bx, by, bz);
    const uint32_t key = launch_key(a);
    // stochastic rounding (DTH; FP32: the dither, 16-bit: at the store): the lane's column
    // word once, a wave-uniform plane word per plane
    constexpr bool DITHER = DTH && std::is_same<T, float>::value;
    const uint32_t colw = DTH ? sr_column(g, gx, gy, key) : 0u;
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        // plane z and its ring into LDS: the side halos of plane z sit at face
        // coordinate v = z, i.e. in the lanes with ly == z (face coordinate u = lx)
#pragma unroll
        for (int s = 0; s < S; ++s) {
            float *ts = tile[wv][s];
            ts[z8::pix(lx, ly)] = c[s][z];
            if (ly == z) {
                ts[z8::pix(-1, lx)] = side[0][s];
                ts[z8::pix(8, lx)] = side[1][s];
                ts[z8::pix(lx, -1)] = side[2][s];
                ts[z8::pix(lx, 8)] = side[3][s];
            }
        }
        // the wave's LDS writes complete before its reads of other lanes' words
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        const int gz = bz * 8 + z;
        // active-neighbour count; walls are the in-box neighbours that are not active
        // (out-of-box ones never are)
        const float nact = (float)((ncw >> (3 * z)) & 7u);
        const bool act = lane_bit(Wo[z]);
        unsigned onf = 0u;
        if (bnd) onf = box_faces(g, gx, gy, gz);
        const float nwall = (6.0f - nact) - (float)__popc(onf);
        float cen[S], res[S];
#pragma unroll
        for (int s = 0; s < S; ++s) cen[s] = c[s][z];
        const uint32_t h = DTH ? sr_combine(colw, sr_plane(gz, key)) : 0u;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const float *p = &tile[wv][s][z8::pix(lx, ly)];
            const float dn = z == 0 ? zlo[s] : c[s][z > 0 ? z - 1 : 0];
            const float up = z == 7 ? zhi[s] : c[s][z < 7 ? z + 1 : 7];
            const float nbv[6] = {p[-1], p[1], p[-10], p[10], dn, up};
            const float dth = DITHER ? fp32_dither(cen[s], sr_species(h, s)) : 0.0f;
            const float upd = rd_update_n<S, DITHER>(cen[s], nbv, nact, nwall, a.coef[s], cen, dth);
            float r = upd;
            if (bnd) {  // Dirichlet voxels lie on the box faces: boundary blocks only (uniform)
                if ((onf & a.coef[s].dir) != 0u) r = cen[s];
            }
            res[s] = act ? r : 0.0f;
        }
        // every lane has read plane z before any lane overwrites it with plane z + 1
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // block-major: whole sectors only (an inactive slot of an active sector stores
        // its 0 again); compact: the active voxels, a contiguous run
        if (lane_bit(CMP ? Wo[z] : sector_lanes<T>(Wo[z]))) {
#pragma unroll
            for (int s = 0; s < S; ++s)
                store_val_ct<T, CMP, DTH>(at_byte(coutb[s], oi[z] * (uint32_t)sizeof(T)), s, 0, h, res[s]);
        }
    }
}

template <typename T, int S, bool XCH, bool CMP, bool DTH>
__global__ __launch_bounds__(256) void k_step8z(StepArgs a)
{
    step8z_group<T, S, XCH, CMP, DTH>(a, map_group(blockIdx.x, a.xcd_chunk));
}

// Several steps in one launch: a cooperative grid, every workgroup resident at once,
// walks the block groups once per step and meets at a grid barrier between steps (a step
// reads what the previous one wrote, possibly on another XCD; the barrier orders those
// writes before the reads and makes them visible).  Each step is k_step8z's per-group
// work with that step's buffers and rounding key, so the fields equal those of one launch
// per step bit for bit.  The memory traffic per step is the same; what goes is the launch
// and its ramp-up and drain per step, which dominate small volumes.  XCD-aware: workgroup
// w runs on XCD w mod 8, and XCD x walks the x-th eighth of the groups.  The grid is a
// multiple of 8 workgroups.
template <typename T, int S, bool XCH, bool DTH>
__global__ __launch_bounds__(256) void k_step8z_fused(StepArgs a, int nsteps)
{
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    const int ngroups = (a.nb + 3) / 4;
    const int per_xcd = (ngroups + 7) / 8;
    const int xcd = (int)blockIdx.x & 7, w = (int)blockIdx.x >> 3, nw = (int)gridDim.x >> 3;
    const int g0 = xcd * per_xcd, g1 = min(g0 + per_xcd, ngroups);
    for (int k = 0; k < nsteps; ++k) {
        StepArgs ak = a;
        if (k & 1) {  // ping-pong
            ak.cin = a.cout;
            ak.cout = const_cast<void *>(a.cin);
        }
        ak.ctr_off = a.ctr_off + (uint32_t)k;
        for (int grp = g0 + w; grp < g1; grp += nw) {
            step8z_group<T, S, XCH, false, DTH>(ak, grp);
            if (XCH) __syncthreads();  // the x-face hand-over arrays serve the next group
        }
        if (k + 1 < nsteps) grid.sync();
    }
}

// ---------------------------------------------------------------------------
// Persistent B = 8 step.  A fixed grid of workgroups walks the block list; while
// block k is computed from LDS, the loads of block k+1 (own slots, halos, mask
// record) are already in flight in registers, so every wave keeps HBM requests
// outstanding across the barrier-compute-store phase.  Thread mapping: wave w
// owns planes lz = 2w, 2w+1; lane l holds the x-adjacent pair lx = 2(l%4), +1 at
// ly = (l/4)%8, lz = 2w + l/32, so own slots move as one 8-byte (FP32) or 4-byte
// (BF16 / FP16) access.  With xcd_chunk > 0, XCD x (= workgroup id mod 8) walks
// the x-th eighth of the list, so +-x / +-y halos are mostly hits in its own L2.
// ---------------------------------------------------------------------------
namespace p8 {
constexpr int TX = 12;            // padded x extent of the LDS tile: [pad, -x, 0..7, +x, pad]
constexpr int TY = 10, TZ = 10;   // y and z extents with halos
constexpr int TL = TX * TY * TZ;  // 1200 words per species
__device__ __forceinline__ int tix(int lx, int ly, int lz)
{
    return ((lz + 1) * TY + (ly + 1)) * TX + (lx + 2);
}
// neighbour-block slot and tile index of face f at face coordinates (u, v)
__device__ __forceinline__ void halo(int f, int u, int v, int *ns, int *t)
{
    switch (f) {
    case 0: *ns = (v * 8 + u) * 8 + 7; *t = tix(-1, u, v); break;
    case 1: *ns = (v * 8 + u) * 8 + 0; *t = tix(8, u, v); break;
    case 2: *ns = (v * 8 + 7) * 8 + u; *t = tix(u, -1, v); break;
    case 3: *ns = (v * 8 + 0) * 8 + u; *t = tix(u, 8, v); break;
    case 4: *ns = (7 * 8 + v) * 8 + u; *t = tix(u, v, -1); break;
    default: *ns = (0 * 8 + v) * 8 + u; *t = tix(u, v, 8); break;
    }
}
template <int S>
struct Regs {
    float c0[S], c1[S], h0[S], h1[S];
    uint64_t mw;
};
}  // namespace p8

// Issue every load of block b for this thread: its own pair, the halo value of face w
// (neighbour n0) and, for waves 0-1, of face 4 + w (neighbour n1); threads 0-15 also
// fetch one word of the mask record.
template <typename T, int S>
__device__ __forceinline__ void p8_load(const StepArgs &a, const T *cin, int b, int n0, int n1,
                                        int w, int slot0, int ns0, int ns1, p8::Regs<S> &r)
{
    const int64_t base = (int64_t)b * 512;
#pragma unroll
    for (int s = 0; s < S; ++s) rd_ld2(cin, s * a.sstride + base + slot0, r.c0[s], r.c1[s]);
    // a missing neighbour reads the block itself (always valid) and selects 0
    const int64_t hb0 = (int64_t)(n0 >= 0 ? n0 : b) * 512 + ns0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const float v = rd_ld(cin, s * a.sstride + hb0);
        r.h0[s] = n0 >= 0 ? v : 0.0f;
    }
    if (w < 2) {
        const int64_t hb1 = (int64_t)(n1 >= 0 ? n1 : b) * 512 + ns1;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const float v = rd_ld(cin, s * a.sstride + hb1);
            r.h1[s] = n1 >= 0 ? v : 0.0f;
        }
    }
    if (threadIdx.x < 16) r.mw = a.mask[(int64_t)b * 16 + threadIdx.x];
}

template <typename T, int S, bool DTH>
__global__ __launch_bounds__(256) void k_step8p(StepArgs a)
{
    __shared__ __align__(16) float tile[S][p8::TL];
    __shared__ uint64_t srec[16];

    // block range of this workgroup
    int64_t lo = 0, hi = a.nb;
    int first = blockIdx.x, stride = gridDim.x;
    if (a.xcd_chunk > 0) {
        const int x = blockIdx.x & 7, per = gridDim.x >> 3;
        lo = (int64_t)a.nb * x / 8;
        hi = (int64_t)a.nb * (x + 1) / 8;
        first = (int)lo + (blockIdx.x >> 3);
        stride = per;
    }
    int b = first;
    if (b >= hi) return;  // uniform: the whole workgroup leaves

    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int lx2 = lane & 3, ly = (lane >> 2) & 7, lzp = 2 * w + (lane >> 5);
    const int slot0 = (lzp * 8 + ly) * 8 + 2 * lx2;
    int ns0, tx0, ns1 = 0, tx1 = 0;
    p8::halo(w, lane & 7, lane >> 3, &ns0, &tx0);
    if (w < 2) p8::halo(4 + w, lane & 7, lane >> 3, &ns1, &tx1);
    const T *cin = (const T *)a.cin;
    T *cout = (T *)a.cout;
    const bool sr = a.sround != 0;
    const uint32_t key = launch_key(a);

    // Block records travel through a double-buffered LDS slot (threads 0-7 hold the
    // next record in a register), which keeps them out of scalar registers.
    __shared__ int32_t sinfo[2][8];
    p8::Regs<S> cur;
    {
        const int32_t *ib = reinterpret_cast<const int32_t *>(a.info + b);
        p8_load<T, S>(a, cin, b, ib[w], w < 2 ? ib[4 + w] : -1, w, slot0, ns0, ns1, cur);
        if (threadIdx.x < 8) sinfo[0][threadIdx.x] = ib[threadIdx.x];
    }
    int bn = b + stride;
    int32_t iw = 0;  // threads 0-7: word threadIdx.x of block bn's record
    if (threadIdx.x < 8 && bn < hi) iw = reinterpret_cast<const int32_t *>(a.info + bn)[threadIdx.x];
    int ph = 0;  // sinfo[ph] holds block b's record

    for (;;) {
        // stage block b (and block bn's record)
#pragma unroll
        for (int s = 0; s < S; ++s) {
            *reinterpret_cast<float2 *>(&tile[s][p8::tix(2 * lx2, ly, lzp)]) =
                make_float2(cur.c0[s], cur.c1[s]);
            tile[s][tx0] = cur.h0[s];
            if (w < 2) tile[s][tx1] = cur.h1[s];
        }
        if (threadIdx.x < 16) srec[threadIdx.x] = cur.mw;
        if (threadIdx.x < 8) sinfo[ph ^ 1][threadIdx.x] = iw;
        __syncthreads();

        // prefetch block bn (and the record of the one after)
        const bool more = bn < hi;
        p8::Regs<S> nxt;
        if (more) {
            const int n0 = sinfo[ph ^ 1][w];
            const int n1 = w < 2 ? sinfo[ph ^ 1][4 + w] : -1;
            p8_load<T, S>(a, cin, bn, n0, n1, w, slot0, ns0, ns1, nxt);
        }
        const int bnn = bn + stride;
        if (threadIdx.x < 8 && more && bnn < hi)
            iw = reinterpret_cast<const int32_t *>(a.info + bnn)[threadIdx.x];

        // compute block b
        int bx, by, bz, gid;
        BlockInfo bi;
        bi.xy = sinfo[ph][6];
        bi.zg = sinfo[ph][7];
        block_pos(bi, &bx, &by, &bz, &gid);
        const GeomInfo g = a.geom[gid];
        const uint64_t W = srec[lzp];
        const uint64_t Wm = lzp > 0 ? srec[lzp - 1] : srec[12];
        const uint64_t Wp = lzp < 7 ? srec[lzp + 1] : srec[13];
        const uint64_t fx0 = srec[8], fx1 = srec[9], fy0 = srec[10], fy1 = srec[11];
        const int gy = by * 8 + ly, gz = bz * 8 + lzp;
        const int64_t base = (int64_t)b * 512;
        float res[2][S];
        const uint32_t h0 = voxel_bits(a, key, g, bx * 8 + 2 * lx2, gy, gz),
                       h1 = voxel_bits(a, key, g, bx * 8 + 2 * lx2 + 1, gy, gz);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int lx = 2 * lx2 + j;
            float cen[S];
#pragma unroll
            for (int s = 0; s < S; ++s) cen[s] = j == 0 ? cur.c0[s] : cur.c1[s];
            vox8<S, DTH>(a, &tile[0][p8::tix(lx, ly, lzp)], p8::TL, p8::TX, p8::TX * p8::TY, W, Wm, Wp,
                         fx0, fx1, fy0, fy1, lx, ly, lzp, box_faces(g, bx * 8 + lx, gy, gz), cen, res[j],
                         j == 0 ? h0 : h1);
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int64_t idx = s * a.sstride + base + slot0;
            rd_st2(cout, idx, res[0][s], res[1][s], sr, sr_species(h0, s), sr_species(h1, s));
        }
        if (!more) break;
        __syncthreads();  // every wave is done with the tile before it is refilled
        cur = nxt;
        b = bn;
        bn = bnn;
        ph ^= 1;
    }
}

// Per-workgroup FP64 balance partials of species a.s:
//   lane 0 mass, lanes 1..6 inflow per Dirichlet face, 7 Robin uptake,
//   8 reaction total, 9 count of non-finite active values.
template <typename T, int B>
__global__ __launch_bounds__(256) void k_reduce(ReduceArgs a)
{
    using K = Blk<B>;
    using C = Cfg<B>;
    __shared__ float tile[C::BPW][1][K::TL];
    __shared__ double wsum[4][RD_NRED];

    const int sub = threadIdx.x / C::TPB;
    const int lt = threadIdx.x % C::TPB;
    const int b = a.b0 + (int)blockIdx.x * C::BPW + sub;
    const bool valid = b < a.b0 + a.nb;
    const T *c = (const T *)a.c;

    BlockInfo bi = {};
    if (valid) bi = a.info[b];
    const T *cs = c + a.s * a.sstride;
    stage_tile<T, B>(tile[sub], cs, 0, 1, b, bi, lt, valid);
    __syncthreads();

    double acc[RD_NRED];
#pragma unroll
    for (int l = 0; l < RD_NRED; ++l) acc[l] = 0.0;
    bool dblock = false;  // the block touches a Dirichlet face of the species
    if (valid) {
        int bx, by, bz, gid;
        block_pos(bi, &bx, &by, &bz, &gid);
        const GeomInfo g = a.geom[gid];
        const bool at[6] = {bx == 0, bx * B + B >= g.nx, by == 0, by * B + B >= g.ny, bz == 0,
                            bz * B + B >= g.nz};
#pragma unroll
        for (int f = 0; f < 6; ++f) dblock = dblock || (((a.dir >> f) & 1u) && at[f]);
        const double dx = a.dx, dx2 = dx * dx, dx3 = dx2 * dx;
#pragma unroll
        for (int k = 0; k < C::VPT; ++k) {
            const int slot = lt + k * C::TPB;
            const int lx = slot % B, ly = (slot / B) % B, lz = slot / (B * B);
            const int gx = bx * B + lx, gy = by * B + ly, gz = bz * B + lz;
            const unsigned code = a.code[(int64_t)b * K::NS + slot];
            if (!(code & 64u)) continue;
            const unsigned nbm = code & 63u;
            const int nwall = __popc(~box_faces(g, gx, gy, gz) & ~nbm & 0x3fu);
            const int t = K::tidx(lx, ly, lz);
            const float *ts = tile[sub][0];
            const double u = (double)ts[t];
            if (!isfinite(ts[t])) acc[9] += 1.0;
            if (on_dirichlet(a.dir, gx, gy, gz, g.nx, g.ny, g.nz)) {
                // first flagged face (in face order) this voxel lies on
                int fq = 0;
                const int onf[6] = {gx == 0, gx == g.nx - 1, gy == 0, gy == g.ny - 1, gz == 0,
                                    gz == g.nz - 1};
                for (int f = 5; f >= 0; --f)
                    if (((a.dir >> f) & 1u) && onf[f]) fq = f;
                const int off[6] = {-1, 1, -K::E, K::E, -K::E * K::E, K::E * K::E};
                const int ddx[6] = {-1, 1, 0, 0, 0, 0}, ddy[6] = {0, 0, -1, 1, 0, 0},
                          ddz[6] = {0, 0, 0, 0, -1, 1};
                double fin = 0.0;
#pragma unroll
                for (int d = 0; d < 6; ++d) {
                    if (!((nbm >> d) & 1u)) continue;
                    if (on_dirichlet(a.dir, gx + ddx[d], gy + ddy[d], gz + ddz[d], g.nx, g.ny, g.nz))
                        continue;
                    fin += a.D * (u - (double)ts[t + off[d]]) * dx;
                }
#pragma unroll
                for (int f = 0; f < 6; ++f)
                    if (f == fq) acc[1 + f] += fin;
                continue;
            }
            acc[0] += u * dx3;
            acc[7] += a.kR * (double)nwall * u * dx2;
            double re = -a.rate_out * u;
            for (int s2 = 0; s2 < a.S; ++s2)
                if (a.rate_in[s2] != 0.0)
                    re += a.rate_in[s2] * (double)rd_ld(c, s2 * a.sstride + (int64_t)b * K::NS + slot);
            acc[8] += re * dx3;
        }
    }
    // wave sums of the lanes that can be nonzero (every flag is uniform per wave: a
    // B = 8 block spans the workgroup, a B = 4 block is one wave); the others are 0
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    bool hasreact = a.rate_out != 0.0;
    for (int s2 = 0; s2 < a.S; ++s2) hasreact = hasreact || a.rate_in[s2] != 0.0;
#pragma unroll
    for (int l = 0; l < RD_NRED; ++l) {
        const bool need = l == 0 || l == 9 || (l <= 6 && dblock) || (l == 7 && a.kR != 0.0) ||
                          (l == 8 && hasreact);
        const double v = need ? wave_sum(acc[l]) : 0.0;
        if (lane == 0) wsum[wave][l] = v;
    }
    __syncthreads();
    if (threadIdx.x < RD_NRED) {
        const int l = threadIdx.x;
        a.partial[(int64_t)blockIdx.x * RD_NRED + l] =
            ((wsum[0][l] + wsum[1][l]) + wsum[2][l]) + wsum[3][l];
    }
}

// The same reduction for 8^3 blocks in the column form of the step: one wave per block,
// four blocks per workgroup, lane (lx, ly) walking its z-column, loads under the
// voxel-activity predicate.  The per-voxel terms are those of k_reduce; a Dirichlet
// voxel (only in blocks on a flagged box face) reads each of its free neighbours
// directly.  One row of RD_NRED partials per workgroup: its four wave sums in wave order.
template <typename T>
__global__ __launch_bounds__(256) void k_reduce8z(ReduceArgs a)
{
    __shared__ double wsum[4][RD_NRED];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int b = __builtin_amdgcn_readfirstlane(a.b0 + (int)blockIdx.x * 4 + wv);
    double acc[RD_NRED];
#pragma unroll
    for (int l = 0; l < RD_NRED; ++l) acc[l] = 0.0;
    bool hasreact = a.rate_out != 0.0;
    for (int s2 = 0; s2 < a.S; ++s2) hasreact = hasreact || a.rate_in[s2] != 0.0;
    bool dblock = false;
    if (b < a.b0 + a.nb) {  // wave-uniform; the barrier below is outside
        const BlockInfo bi = a.info[b];
        int bx, by, bz, gid;
        block_pos(bi, &bx, &by, &bz, &gid);
        const GeomInfo g = a.geom[gid];
        const uint64_t *rec = a.mask + (int64_t)b * 16;
        const int64_t base = (int64_t)b * 512;
        const T *c = (const T *)a.c;
        const T *cs = c + a.s * a.sstride;
        const int lx = lane & 7, ly = lane >> 3;
        const int gx = bx * 8 + lx, gy = by * 8 + ly;
        const bool at[6] = {bx == 0, bx * 8 + 8 >= g.nx, by == 0, by * 8 + 8 >= g.ny, bz == 0,
                            bz * 8 + 8 >= g.nz};
        bool bnd = false;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            bnd = bnd || at[f];
            dblock = dblock || (((a.dir >> f) & 1u) && at[f]);
        }
        typedef typename RawOf<T>::type R;
        uint64_t Wo[8];
        R raw[8];
        unsigned cd[8];
        int64_t oi[8];  // element index of the lane's voxel in plane z (block-major or compact)
        int64_t acc0 = a.cbase ? (int64_t)a.cbase[b] : 0;
#pragma unroll
        for (int z = 0; z < 8; ++z) {
            Wo[z] = rec[z];
            oi[z] = a.cbase ? acc0 + lanes_below(Wo[z]) : base + z * 64 + lane;
            acc0 += __popcll(Wo[z]);
            const bool act = (Wo[z] >> lane) & 1ull;
            raw[z] = ld_raw(cs, oi[z], act);
            cd[z] = act ? (unsigned)a.code[oi[z]] : 0u;
        }
        // inflow into this species from the others (0 on inactive slots)
        double rin[8];
#pragma unroll
        for (int z = 0; z < 8; ++z) rin[z] = 0.0;
        for (int s2 = 0; s2 < a.S; ++s2) {
            const double k = a.rate_in[s2];
            if (k == 0.0) continue;
            R r2[8];
#pragma unroll
            for (int z = 0; z < 8; ++z) r2[z] = ld_raw(c + s2 * a.sstride, oi[z], (Wo[z] >> lane) & 1ull);
#pragma unroll
            for (int z = 0; z < 8; ++z) rin[z] += k * (double)from_raw<T>(r2[z]);
        }
        const double dx = a.dx, dx2 = dx * dx, dx3 = dx2 * dx;
#pragma unroll
        for (int z = 0; z < 8; ++z) {
            const unsigned code = cd[z];
            if (!(code & 64u)) continue;
            const float uf = from_raw<T>(raw[z]);
            const double u = (double)uf;
            if (!isfinite(uf)) acc[9] += 1.0;
            const int gz = bz * 8 + z;
            const unsigned onf = bnd ? box_faces(g, gx, gy, gz) : 0u;
            if (onf & a.dir) {
                // Dirichlet voxel: inflow into its free neighbours, booked on the first
                // flagged face (in face order) it lies on
                const int fq = __builtin_ctz(onf & a.dir);
                double fin = 0.0;
#pragma unroll
                for (int d = 0; d < 6; ++d) {
                    if (!((code >> d) & 1u)) continue;
                    const int ex = d == 0 ? -1 : d == 1 ? 1 : 0;
                    const int ey = d == 2 ? -1 : d == 3 ? 1 : 0;
                    const int ez = d == 4 ? -1 : d == 5 ? 1 : 0;
                    if (on_dirichlet(a.dir, gx + ex, gy + ey, gz + ez, g.nx, g.ny, g.nz)) continue;
                    const int qx = lx + ex, qy = ly + ey, qz = z + ez;
                    const bool inside = qx >= 0 && qx < 8 && qy >= 0 && qy < 8 && qz >= 0 && qz < 8;
                    // an active neighbour outside the block lies in face neighbour d
                    const int nbk = inside ? b : bi.nbr[d];
                    const int slot = ((qz & 7) * 8 + (qy & 7)) * 8 + (qx & 7);
                    const double v = (double)rd_ld(cs, slot_index8(a.cbase, a.mask, nbk, slot));
                    fin += a.D * (u - v) * dx;
                }
#pragma unroll
                for (int f = 0; f < 6; ++f)
                    if (f == fq) acc[1 + f] += fin;
                continue;
            }
            acc[0] += u * dx3;
            if (a.kR != 0.0) {
                const int nwall = __popc(~onf & ~code & 0x3fu);
                acc[7] += a.kR * (double)nwall * u * dx2;
            }
            if (hasreact) acc[8] += (rin[z] - a.rate_out * u) * dx3;
        }
    }
#pragma unroll
    for (int l = 0; l < RD_NRED; ++l) {
        const bool need = l == 0 || l == 9 || (l <= 6 && dblock) || (l == 7 && a.kR != 0.0) ||
                          (l == 8 && hasreact);
        const double v = need ? wave_sum(acc[l]) : 0.0;
        if (lane == 0) wsum[wv][l] = v;
    }
    __syncthreads();
    if (threadIdx.x < RD_NRED) {
        const int l = threadIdx.x;
        a.partial[(int64_t)blockIdx.x * RD_NRED + l] =
            ((wsum[0][l] + wsum[1][l]) + wsum[2][l]) + wsum[3][l];
    }
}

// Diffusive flux of one species through the plane between indices i0 and i0 + 1 along
// `axis`: sum over pairs (p, p + e_axis) of active voxels of D (c_p - c_{p+e}) dx.  One
// wave per block, four blocks per workgroup; lane l < B^2 takes in-plane position l of
// the block's layer i0, if the block holds it.  One FP64 partial per workgroup (its
// four wave sums in wave order).
template <typename T, int B>
__global__ __launch_bounds__(256) void k_plane_flux(const BlockInfo *info, const uint8_t *code,
                                                    const uint32_t *cbase, const uint64_t *mask,
                                                    const T *c, int nb, int axis, int i0,
                                                    double D, double dx, double *partial)
{
    using K = Blk<B>;
    __shared__ double wsum[4];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int b = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + wv);
    double q = 0.0;
    if (b < nb) {
        const BlockInfo bi = info[b];
        int bx, by, bz, gid;
        block_pos(bi, &bx, &by, &bz, &gid);
        const int l0 = i0 - (axis == 0 ? bx : axis == 1 ? by : bz) * B;
        if (l0 >= 0 && l0 < B && lane < B * B) {
            const int u = lane % B, v = lane / B;
            const int lx = axis == 0 ? l0 : u, ly = axis == 1 ? l0 : axis == 0 ? u : v,
                      lz = axis == 2 ? l0 : v;
            const int slot = (lz * B + ly) * B + lx;
            const int stride = axis == 0 ? 1 : axis == 1 ? B : B * B;
            // compact layout (B = 8 only): the slot's code and value exist only if it is
            // active
            const bool own = !cbase || own_bit<B>(mask + (int64_t)b * K::MW, slot);
            const int64_t ip = cbase ? slot_index8(cbase, mask, b, slot) : (int64_t)b * K::NS + slot;
            const unsigned cd = own ? code[ip] : 0u;
            if ((cd & 64u) && ((cd >> (2 * axis + 1)) & 1u)) {
                // the active +axis neighbour is in this block or in face neighbour 2 axis + 1
                const int nbk = l0 + 1 < B ? b : bi.nbr[2 * axis + 1];
                const int ns = l0 + 1 < B ? slot + stride : slot - (B - 1) * stride;
                const int64_t iq = cbase ? slot_index8(cbase, mask, nbk, ns) : (int64_t)nbk * K::NS + ns;
                const double cp = (double)rd_ld(c, ip);
                const double cq = (double)rd_ld(c, iq);
                q = D * (cp - cq) * dx;
            }
        }
    }
    const double s = wave_sum(q);
    if (lane == 0) wsum[wv] = s;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
}

// Row sums of a [nrows][nlanes] FP64 array (nlanes <= RD_FINISH_LANES): workgroup g
// sums rows [g * chunk, min((g + 1) * chunk, nrows)) into out[g][*].  Thread t adds
// rows t, t + 256, ... of the range (whole rows, so loads are coalesced), then a
// fixed tree over the threads; the order depends only on nrows and chunk.
#define RD_FINISH_LANES 16
__global__ __launch_bounds__(256) void k_finish_rows(const double *part, int nrows, int nlanes,
                                                     int chunk, double *out)
{
    __shared__ double sh[RD_FINISH_LANES][257];
    const int g = blockIdx.x, t = threadIdx.x;
    const int64_t r0 = (int64_t)g * chunk;
    const int64_t r1 = r0 + chunk < nrows ? r0 + chunk : nrows;
    double acc[RD_FINISH_LANES];
#pragma unroll
    for (int l = 0; l < RD_FINISH_LANES; ++l) acc[l] = 0.0;
    for (int64_t r = r0 + t; r < r1; r += 256) {
#pragma unroll
        for (int l = 0; l < RD_FINISH_LANES; ++l)
            if (l < nlanes) acc[l] += part[r * nlanes + l];
    }
#pragma unroll
    for (int l = 0; l < RD_FINISH_LANES; ++l) sh[l][t] = acc[l];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
#pragma unroll
            for (int l = 0; l < RD_FINISH_LANES; ++l) sh[l][t] += sh[l][t + w];
        }
        __syncthreads();
    }
    if (t < nlanes) out[(int64_t)g * nlanes + t] = sh[t][0];
}

// Dense float32 -> block-major storage of one species.  Inactive slots get 0 and
// Dirichlet voxels their held value (the highest flagged face wins on shared edges).
template <typename T, int B>
__global__ __launch_bounds__(256) void k_scatter(const BlockInfo *info, const uint64_t *mask,
                                                 const uint32_t *cbase, const GeomInfo *geom, int nb,
                                                 const float *dense, T *field, uint32_t dir, float d0,
                                                 float d1, float d2, float d3, float d4, float d5)
{
    using K = Blk<B>;
    const int b = blockIdx.x;
    if (b >= nb) return;
    const BlockInfo bi = info[b];
    int bx, by, bz, gid;
    block_pos(bi, &bx, &by, &bz, &gid);
    const GeomInfo g = geom[gid];
    const uint64_t *rec = mask + (int64_t)b * K::MW;
    const float dv[6] = {d0, d1, d2, d3, d4, d5};
    for (int slot = threadIdx.x; slot < K::NS; slot += 256) {
        const int lx = slot % B, ly = (slot / B) % B, lz = slot / (B * B);
        const int gx = bx * B + lx, gy = by * B + ly, gz = bz * B + lz;
        float v = 0.0f;
        const bool own = own_bit<B>(rec, slot);
        if (own) {
            v = dense[voxel_id(g, gx, gy, gz)];
            const int onf[6] = {gx == 0, gx == g.nx - 1, gy == 0, gy == g.ny - 1, gz == 0,
                                gz == g.nz - 1};
            for (int f = 0; f < 6; ++f)
                if (((dir >> f) & 1u) && onf[f]) v = dv[f];
        }
        // compact layout: only active voxels are stored
        if (!cbase) rd_st(field, (int64_t)b * K::NS + slot, v);
        else if (own) rd_st(field, slot_index8(cbase, mask, b, slot), v);
    }
}

// Block-major storage -> dense float32 (active voxels only; the caller zero-fills).
template <typename T, int B>
__global__ __launch_bounds__(256) void k_gather(const BlockInfo *info, const uint64_t *mask,
                                                const uint32_t *cbase, const GeomInfo *geom, int nb,
                                                const T *field, float *dense)
{
    using K = Blk<B>;
    const int b = blockIdx.x;
    if (b >= nb) return;
    const BlockInfo bi = info[b];
    int bx, by, bz, gid;
    block_pos(bi, &bx, &by, &bz, &gid);
    const GeomInfo g = geom[gid];
    const uint64_t *rec = mask + (int64_t)b * K::MW;
    for (int slot = threadIdx.x; slot < K::NS; slot += 256) {
        if (!own_bit<B>(rec, slot)) continue;
        const int lx = slot % B, ly = (slot / B) % B, lz = slot / (B * B);
        const int gx = bx * B + lx, gy = by * B + ly, gz = bz * B + lz;
        const int64_t i = cbase ? slot_index8(cbase, mask, b, slot) : (int64_t)b * K::NS + slot;
        dense[voxel_id(g, gx, gy, gz)] = rd_ld(field, i);
    }
}

// Set the Dirichlet voxels of one species in a block-major field (others untouched).
template <typename T, int B>
__global__ __launch_bounds__(256) void k_set_dirichlet(const BlockInfo *info, const uint64_t *mask,
                                                       const uint32_t *cbase, const GeomInfo *geom,
                                                       int nb, T *field, uint32_t dir, float d0,
                                                       float d1, float d2, float d3, float d4,
                                                       float d5)
{
    using K = Blk<B>;
    const int b = blockIdx.x;
    if (b >= nb) return;
    const BlockInfo bi = info[b];
    int bx, by, bz, gid;
    block_pos(bi, &bx, &by, &bz, &gid);
    const GeomInfo g = geom[gid];
    const uint64_t *rec = mask + (int64_t)b * K::MW;
    const float dv[6] = {d0, d1, d2, d3, d4, d5};
    for (int slot = threadIdx.x; slot < K::NS; slot += 256) {
        if (!own_bit<B>(rec, slot)) continue;
        const int lx = slot % B, ly = (slot / B) % B, lz = slot / (B * B);
        const int gx = bx * B + lx, gy = by * B + ly, gz = bz * B + lz;
        const int onf[6] = {gx == 0, gx == g.nx - 1, gy == 0, gy == g.ny - 1, gz == 0,
                            gz == g.nz - 1};
        bool hit = false;
        float v = 0.0f;
        for (int f = 0; f < 6; ++f)
            if (((dir >> f) & 1u) && onf[f]) { v = dv[f]; hit = true; }
        if (hit) rd_st(field, cbase ? slot_index8(cbase, mask, b, slot) : (int64_t)b * K::NS + slot, v);
    }
}

__global__ void k_add_u32(uint32_t *p, uint32_t add)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = p[0] + add;
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *p, uint32_t v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        p[i] = v;
}

template <int B>
int groups_for(int nb) { return (nb + Cfg<B>::BPW - 1) / Cfg<B>::BPW; }

// SR: stochastic rounding on.  The column kernel takes it for every storage type (FP32:
// the dither; 16-bit: the rounding of its stores, fixed at compile time); the other
// kernels take it as the FP32 dither only and round 16-bit stores by the run-time flag.
template <typename T, int B, int S, bool SR>
void launch_step_d(const StepArgs &a, int groups, hipStream_t st)
{
    constexpr bool DTH = SR && std::is_same<T, float>::value;
    if constexpr (B == 8) {
        if (a.kernel == 1)
            hipLaunchKernelGGL((k_step8p<T, S, DTH>), dim3(a.grid), dim3(256), 0, st, a);
        else if (a.kernel == 2 && a.cbase)
            hipLaunchKernelGGL((k_step8z<T, S, false, true, SR>), dim3(groups), dim3(256), 0, st, a);
        else if (a.kernel == 3 && a.cbase)
            hipLaunchKernelGGL((k_step8z<T, S, true, true, SR>), dim3(groups), dim3(256), 0, st, a);
        else if (a.kernel == 2)
            hipLaunchKernelGGL((k_step8z<T, S, false, false, SR>), dim3(groups), dim3(256), 0, st, a);
        else if (a.kernel == 3)
            hipLaunchKernelGGL((k_step8z<T, S, true, false, SR>), dim3(groups), dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL((k_step8<T, S, DTH>), dim3(groups), dim3(256), 0, st, a);
    } else {
        hipLaunchKernelGGL((k_step4w<T, S, DTH>), dim3(groups), dim3(256), 0, st, a);
    }
}

// FP32 storage with stochastic rounding runs the dithered kernels; 16-bit storage rounds
// stochastically when it stores.
template <typename T, int B, int S>
void launch_step_s(const StepArgs &a, int groups, hipStream_t st)
{
    if (a.sround) launch_step_d<T, B, S, true>(a, groups, st);
    else launch_step_d<T, B, S, false>(a, groups, st);
}

template <typename T, int B>
int launch_step_t(const StepArgs &a, hipStream_t st)
{
    // blocks per workgroup: 1 for the B = 8 workgroup kernel, 4 for the wave kernels
    const int bpw = (B == 8 && a.kernel < 2) ? 1 : 4;
    int groups = (a.nb + bpw - 1) / bpw;
    if (a.xcd_chunk > 0) groups = 8 * a.xcd_chunk;
    switch (a.S) {
    case 1: launch_step_s<T, B, 1>(a, groups, st); break;
    case 2: launch_step_s<T, B, 2>(a, groups, st); break;
    case 3: launch_step_s<T, B, 3>(a, groups, st); break;
    default: launch_step_s<T, B, 4>(a, groups, st); break;
    }
    return (int)hipGetLastError();
}

template <typename T, int B>
int launch_reduce_t(const ReduceArgs &a, hipStream_t st)
{
    if (B == 8)  // column form, four blocks per workgroup
        hipLaunchKernelGGL((k_reduce8z<T>), dim3(rd_reduce_rows(B, a.nb)), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_reduce<T, B>), dim3(rd_reduce_rows(B, a.nb)), dim3(256), 0, st, a);
    return (int)hipGetLastError();
}

}  // namespace

#define RD_DISPATCH(storage, B, FN, ...)                                     \
    do {                                                                     \
        if ((B) == 8) {                                                      \
            if ((storage) == 0) return FN<float, 8>(__VA_ARGS__);            \
            if ((storage) == 1) return FN<bf16_t, 8>(__VA_ARGS__);           \
            return FN<_Float16, 8>(__VA_ARGS__);                             \
        } else {                                                             \
            if ((storage) == 0) return FN<float, 4>(__VA_ARGS__);            \
            if ((storage) == 1) return FN<bf16_t, 4>(__VA_ARGS__);           \
            return FN<_Float16, 4>(__VA_ARGS__);                             \
        }                                                                    \
    } while (0)

int rd_launch_step(int storage, int B, const StepArgs &a, void *stream)
{
    if (a.nb <= 0) return 0;
    RD_DISPATCH(storage, B, launch_step_t, a, (hipStream_t)stream);
}

namespace {
template <typename T, int S, bool XCH, bool DTH>
int launch_fused_k(const StepArgs &a, int nsteps, int n_cu, hipStream_t st)
{
    const void *fn = (const void *)k_step8z_fused<T, S, XCH, DTH>;
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0);
    if (e != hipSuccess) return (int)e;
    const int ngroups = (a.nb + 3) / 4;
    int grid = per_cu * n_cu;                         // every workgroup resident
    grid = std::min(grid, ((ngroups + 7) / 8) * 8);   // no more than the groups need
    grid = (grid / 8) * 8;
    if (grid < 8) return (int)hipErrorCooperativeLaunchTooLarge;
    StepArgs args = a;
    int ns = nsteps;
    void *params[] = {(void *)&args, (void *)&ns};
    return (int)hipLaunchCooperativeKernel(fn, dim3((unsigned)grid), dim3(256), params, 0, st);
}
template <typename T, int S>
int launch_fused_s(const StepArgs &a, int nsteps, int n_cu, hipStream_t st)
{
    const bool xch = a.kernel == 3, sr = a.sround != 0;
    if (xch) return sr ? launch_fused_k<T, S, true, true>(a, nsteps, n_cu, st)
                       : launch_fused_k<T, S, true, false>(a, nsteps, n_cu, st);
    return sr ? launch_fused_k<T, S, false, true>(a, nsteps, n_cu, st)
              : launch_fused_k<T, S, false, false>(a, nsteps, n_cu, st);
}
template <typename T>
int launch_fused_t(const StepArgs &a, int nsteps, int n_cu, hipStream_t st)
{
    switch (a.S) {
    case 1: return launch_fused_s<T, 1>(a, nsteps, n_cu, st);
    case 2: return launch_fused_s<T, 2>(a, nsteps, n_cu, st);
    case 3: return launch_fused_s<T, 3>(a, nsteps, n_cu, st);
    default: return launch_fused_s<T, 4>(a, nsteps, n_cu, st);
    }
}
}  // namespace

int rd_launch_step_fused(int storage, const StepArgs &a, int nsteps, int n_cu, void *stream)
{
    if (a.nb <= 0 || nsteps <= 0) return 0;
    if (storage == 0) return launch_fused_t<float>(a, nsteps, n_cu, (hipStream_t)stream);
    if (storage == 1) return launch_fused_t<bf16_t>(a, nsteps, n_cu, (hipStream_t)stream);
    return launch_fused_t<_Float16>(a, nsteps, n_cu, (hipStream_t)stream);
}

int rd_reduce_rows(int, int nb) { return (nb + 3) / 4; }

namespace {
template <typename T, int B>
int launch_plane_flux_t(const BlockInfo *info, const uint8_t *code, const uint32_t *cbase,
                        const uint64_t *mask, const void *c, int nb, int axis, int i0, double D, double dx,
                        double *partial, hipStream_t st)
{
    hipLaunchKernelGGL((k_plane_flux<T, B>), dim3(rd_reduce_rows(B, nb)), dim3(256), 0, st, info, code,
                       cbase, mask, (const T *)c, nb, axis, i0, D, dx, partial);
    return (int)hipGetLastError();
}
}  // namespace

int rd_launch_plane_flux(int storage, int B, const BlockInfo *info, const uint8_t *code,
                         const uint32_t *cbase, const uint64_t *mask, const void *c, int nb, int axis,
                         int i0, double D, double dx, double *partial, void *stream)
{
    if (nb <= 0) return 0;
    RD_DISPATCH(storage, B, launch_plane_flux_t, info, code, cbase, mask, c, nb, axis, i0, D, dx, partial,
                (hipStream_t)stream);
}

int rd_launch_reduce(int storage, int B, const ReduceArgs &a, void *stream)
{
    if (a.nb <= 0) return 0;
    RD_DISPATCH(storage, B, launch_reduce_t, a, (hipStream_t)stream);
}

int rd_launch_finish_reduce(const double *partial, int nparts, int nlanes, double *mid, double *out,
                            void *stream)
{
    if (nlanes < 1 || nlanes > RD_FINISH_LANES) return (int)hipErrorInvalidValue;
    hipStream_t st = (hipStream_t)stream;
    if (nparts <= 4096) {  // one workgroup in one pass
        hipLaunchKernelGGL(k_finish_rows, dim3(1), dim3(256), 0, st, partial, nparts, nlanes,
                           nparts > 0 ? nparts : 1, out);
        return (int)hipGetLastError();
    }
    // RD_FINISH_GROUPS fixed ranges, then their sums in one workgroup
    const int chunk = (nparts + RD_FINISH_GROUPS - 1) / RD_FINISH_GROUPS;
    const int groups = (nparts + chunk - 1) / chunk;
    hipLaunchKernelGGL(k_finish_rows, dim3(groups), dim3(256), 0, st, partial, nparts, nlanes, chunk,
                       mid);
    hipLaunchKernelGGL(k_finish_rows, dim3(1), dim3(256), 0, st, (const double *)mid, groups, nlanes,
                       groups, out);
    return (int)hipGetLastError();
}

namespace {
template <typename T, int B>
int launch_scatter_t(const BlockInfo *info, const uint64_t *mask, const uint32_t *cbase, const GeomInfo *geom,
                     int nb, const float *dense, void *field, uint32_t dir, const float *dv, hipStream_t st)
{
    hipLaunchKernelGGL((k_scatter<T, B>), dim3(nb), dim3(256), 0, st, info, mask, cbase, geom, nb, dense,
                       (T *)field, dir, dv[0], dv[1], dv[2], dv[3], dv[4], dv[5]);
    return (int)hipGetLastError();
}
template <typename T, int B>
int launch_gather_t(const BlockInfo *info, const uint64_t *mask, const uint32_t *cbase, const GeomInfo *geom,
                    int nb, const void *field, float *dense, hipStream_t st)
{
    hipLaunchKernelGGL((k_gather<T, B>), dim3(nb), dim3(256), 0, st, info, mask, cbase, geom, nb,
                       (const T *)field, dense);
    return (int)hipGetLastError();
}
}  // namespace

int rd_launch_scatter(int storage, int B, const BlockInfo *info, const uint64_t *mask,
                      const uint32_t *cbase, const GeomInfo *geom, int nb, const float *dense, void *field,
                      uint32_t dir, float dir_value_per_face[6], void *stream)
{
    if (nb <= 0) return 0;
    RD_DISPATCH(storage, B, launch_scatter_t, info, mask, cbase, geom, nb, dense, field, dir,
                dir_value_per_face, (hipStream_t)stream);
}

int rd_launch_gather(int storage, int B, const BlockInfo *info, const uint64_t *mask,
                     const uint32_t *cbase, const GeomInfo *geom, int nb, const void *field, float *dense,
                     int64_t ndense, void *stream)
{
    int rc = rd_launch_fill_u32(dense, 0u, ndense, stream);
    if (rc || nb <= 0) return rc;
    RD_DISPATCH(storage, B, launch_gather_t, info, mask, cbase, geom, nb, field, dense,
                (hipStream_t)stream);
}

namespace {
template <typename T, int B>
int launch_setdir_t(const BlockInfo *info, const uint64_t *mask, const uint32_t *cbase, const GeomInfo *geom,
                    int nb, void *field, uint32_t dir, const float *dv, hipStream_t st)
{
    hipLaunchKernelGGL((k_set_dirichlet<T, B>), dim3(nb), dim3(256), 0, st, info, mask, cbase, geom, nb,
                       (T *)field, dir, dv[0], dv[1], dv[2], dv[3], dv[4], dv[5]);
    return (int)hipGetLastError();
}
}  // namespace

int rd_launch_set_dirichlet(int storage, int B, const BlockInfo *info, const uint64_t *mask,
                            const uint32_t *cbase, const GeomInfo *geom, int nb, void *field, uint32_t dir,
                            const float dv[6], void *stream)
{
    if (nb <= 0) return 0;
    RD_DISPATCH(storage, B, launch_setdir_t, info, mask, cbase, geom, nb, field, dir, dv,
                (hipStream_t)stream);
}

int rd_launch_add_u32(uint32_t *ptr, uint32_t add, void *stream)
{
    hipLaunchKernelGGL(k_add_u32, dim3(1), dim3(64), 0, (hipStream_t)stream, ptr, add);
    return (int)hipGetLastError();
}

// Compact layout: the halo record of each block, 32 words: [v] one past the last voxel of
// plane v of the -y neighbour, [8 + v] the first voxel of plane v of the +y neighbour,
// [16] one past the last voxel of the -z neighbour, [17] the first voxel of the +z
// neighbour (0 where there is no neighbour; the rest 0).  One thread per block.
__global__ void k_halo_rec8(const BlockInfo *__restrict__ info, const uint64_t *__restrict__ mask,
                            const uint32_t *__restrict__ cbase, uint32_t *__restrict__ hrec, int nb)
{
    const int b = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (b >= nb) return;
    const BlockInfo bi = info[b];
    const int n2 = bi.nbr[2], n3 = bi.nbr[3], n4 = bi.nbr[4], n5 = bi.nbr[5];
    uint32_t *out = hrec + (int64_t)b * 32;
    for (int v = 0; v < 8; ++v) {
        out[v] = n2 < 0 ? 0u : (v < 7 ? cbase[n2] + plane_prefix(mask + (int64_t)n2 * 16, v + 1) : cbase[n2 + 1]);
        out[8 + v] = n3 < 0 ? 0u : cbase[n3] + plane_prefix(mask + (int64_t)n3 * 16, v);
    }
    out[16] = n4 < 0 ? 0u : cbase[n4 + 1];
    out[17] = n5 < 0 ? 0u : cbase[n5];
    for (int i = 18; i < 32; ++i) out[i] = 0u;
}

int rd_launch_halo_rec8(const BlockInfo *info, const uint64_t *mask, const uint32_t *cbase, uint32_t *hrec,
                        int nb, void *stream)
{
    if (nb <= 0) return 0;
    hipLaunchKernelGGL(k_halo_rec8, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, (hipStream_t)stream, info,
                       mask, cbase, hrec, nb);
    return (int)hipGetLastError();
}

int rd_launch_count_words8(const uint64_t *mask, uint32_t *ncnt, int nb, void *stream)
{
    const int64_t n = (int64_t)nb * 64;
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_count_words8, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, mask,
                       ncnt, n);
    return (int)hipGetLastError();
}

int rd_launch_fill_u32(void *ptr, uint32_t value, int64_t n_words, void *stream)
{
    if (n_words <= 0) return 0;
    int64_t g = (n_words + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)g), dim3(256), 0, (hipStream_t)stream,
                       (uint32_t *)ptr, value, n_words);
    return (int)hipGetLastError();
}
