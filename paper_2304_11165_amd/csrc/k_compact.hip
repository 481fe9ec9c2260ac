// k_compact.hip -- the FTCS step on the compact layout with lane-exchanged neighbours
// (gfx950, wave64).
//
// Same update as every other step kernel (rd_update: paper section "Discretization and
// numerical methods", FTCS with the mirror rule; blocks of 8^3 as in section "Parallel
// implementation using OpenFPM"), so the fields are bitwise those of the block layout.
// What differs is how a wave finds its data:
//   * one wave per block, four blocks per workgroup, lane (lx, ly) walking its z-column;
//   * the block stores only its active voxels (compact layout): plane z starts at
//     cbase[b] + (active slots below z) and a lane's voxel sits at the number of active
//     lanes below it (mbcnt of the plane word), so a plane is one contiguous run;
//   * every access is a buffer access with a 32-bit byte offset: inactive lanes get an
//     offset past the buffer, so their loads return 0 (the value an inactive neighbour
//     contributes) and their stores are dropped -- no per-load predicates, no zeroing;
//   * +-z neighbours are the lane's own registers; -x / +x come from the lane beside it
//     in the row of eight (DPP row shift), -y / +y from the row above / below
//     (ds_bpermute); the face halos of the four side neighbours are loaded once per
//     block in face coordinates (lane (u, v)) and moved to the lanes on the block face
//     plane by plane with ds_bpermute.  No LDS tile, no barrier.
// HBM-bound (about 2 FLOP per byte): no MFMA.
#include "rd_device.h"

namespace {

typedef __amdgpu_buffer_rsrc_t Rsrc;

// A byte offset past every buffer (sizes are checked on the host to stay below it).
constexpr uint32_t OOB = 0xFFFFFFF0u;

__device__ __forceinline__ Rsrc make_rsrc(const void *p, uint32_t bytes)
{
    // raw buffer (stride 0): an access is out of range when its offset reaches `bytes`
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

template <typename T> struct Buf;
template <> struct Buf<float> {
    static constexpr uint32_t ES = 4;
    __device__ static __forceinline__ float ld(Rsrc r, uint32_t off)
    {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
    }
    __device__ static __forceinline__ void st(Rsrc r, uint32_t off, float v, bool, uint32_t)
    {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, 0);
    }
};
template <> struct Buf<bf16_t> {
    static constexpr uint32_t ES = 2;
    __device__ static __forceinline__ uint32_t ld(Rsrc r, uint32_t off)
    {
        return (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
    }
    __device__ static __forceinline__ void st(Rsrc r, uint32_t off, float v, bool sr, uint32_t rnd)
    {
        const uint16_t h = sr ? bf16_sr(v, rnd) : bf16_rne(v);
        __builtin_amdgcn_raw_buffer_store_b16(h, r, off, 0, 0);
    }
};
template <> struct Buf<_Float16> {
    static constexpr uint32_t ES = 2;
    __device__ static __forceinline__ uint32_t ld(Rsrc r, uint32_t off)
    {
        return (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
    }
    __device__ static __forceinline__ void st(Rsrc r, uint32_t off, float v, bool sr, uint32_t rnd)
    {
        const _Float16 h = sr ? f16_sr(v, rnd) : (_Float16)v;
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, h), r, off, 0, 0);
    }
};

// Value of the lane `sh` places to the left (sh > 0: row_shr) or right (sh < 0:
// row_shl) inside its DPP row of 16 lanes, 0 where that lane is outside the row.
template <int SH>
__device__ __forceinline__ float row_shift(float v)
{
    constexpr int ctrl = SH > 0 ? 0x110 + SH : 0x100 - SH;
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), ctrl, 0xf, 0xf, true));
}
__device__ __forceinline__ float lane_read(int byte_addr, float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(byte_addr, __builtin_bit_cast(int, v)));
}

// Element index (in the neighbour's compact run) of the slot across side face f
// (0..3: -x, +x, -y, +y) at face coordinates (u, v) = (lx, ly): the neighbour slot is
// in plane v; its rank is the neighbour's prefix of plane v plus the active slots
// below it in that plane.
__device__ __forceinline__ uint32_t side_index(const StepArgs &a, int f, int nn, int lx, int ly)
{
    const uint64_t *nrec = a.mask + (int64_t)nn * 16;
    const uint64_t nw = nrec[ly];
    const int bit = f == 0 ? lx * 8 + 7 : f == 1 ? lx * 8 : f == 2 ? 56 + lx : lx;
    const uint64_t below = nw & ((1ull << bit) - 1ull);
    return a.cbase[nn] + plane_prefix(nrec, ly) + (uint32_t)__popcll(below);
}

template <typename T, int S, bool DTH>
__global__ __launch_bounds__(256) void k_step8l(StepArgs a)
{
    typedef Buf<T> Bt;
    typedef typename RawOf<T>::type R;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int grp = map_group(blockIdx.x, a.xcd_chunk);
    const int b = __builtin_amdgcn_readfirstlane(grp * 4 + wv);
    if (b >= a.nb) return;
    const int lx = lane & 7, ly = lane >> 3;
    const uint32_t bytes = (uint32_t)((uint64_t)a.sstride * Bt::ES);
    Rsrc rin[S], rout[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        rin[s] = make_rsrc((const T *)a.cin + s * a.sstride, bytes);
        rout[s] = make_rsrc((T *)a.cout + s * a.sstride, bytes);
    }
    const Rsrc rcode = make_rsrc(a.code, (uint32_t)a.sstride);

    const uint64_t *rec = a.mask + (int64_t)b * 16;
    uint64_t Wo[8], Wf[6];
#pragma unroll
    for (int z = 0; z < 8; ++z) Wo[z] = rec[z];
#pragma unroll
    for (int f = 0; f < 6; ++f) Wf[f] = rec[8 + f];

    // byte offsets of the lane's voxel in each plane (OOB where it is inactive)
    uint32_t vo[8], co[8];
    {
        uint32_t acc = a.cbase[b];
#pragma unroll
        for (int z = 0; z < 8; ++z) {
            const uint32_t idx = __builtin_amdgcn_mbcnt_hi((uint32_t)(Wo[z] >> 32),
                                                           __builtin_amdgcn_mbcnt_lo((uint32_t)Wo[z], acc));
            const bool on = lane_bit(Wo[z]);
            co[z] = on ? idx : OOB;
            vo[z] = on ? idx * Bt::ES : OOB;
            acc += (uint32_t)__popcll(Wo[z]);
        }
    }
    R rc[S][8];
    uint32_t cd[8];
#pragma unroll
    for (int z = 0; z < 8; ++z) {
#pragma unroll
        for (int s = 0; s < S; ++s) rc[s][z] = Bt::ld(rin[s], vo[z]);
        cd[z] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(rcode, co[z], 0, 0);
    }
    // face halos in face coordinates: lane (u, v) = (lx, ly) holds the neighbour voxel
    // across face f at (u, v); 0 where it is inactive or missing (face bit clear)
    const int32_t *nbr = a.info[b].nbr;
    R rh[6][S];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const int n = nbr[f];
        const int nn = n >= 0 ? n : b;
        uint32_t idx;
        if (f == 4) {  // plane 7 of the -z neighbour: the last popc(Wf[4]) voxels of its run
            const uint32_t top = a.cbase[nn + 1] - (uint32_t)__popcll(Wf[4]);
            idx = __builtin_amdgcn_mbcnt_hi((uint32_t)(Wf[4] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)Wf[4], top));
        } else if (f == 5) {  // plane 0 of the +z neighbour: the start of its run
            idx = __builtin_amdgcn_mbcnt_hi((uint32_t)(Wf[5] >> 32),
                                            __builtin_amdgcn_mbcnt_lo((uint32_t)Wf[5], a.cbase[nn]));
        } else {
            idx = side_index(a, f, nn, lx, ly);
        }
        const uint32_t ho = lane_bit(Wf[f]) ? idx * Bt::ES : OOB;
#pragma unroll
        for (int s = 0; s < S; ++s) rh[f][s] = Bt::ld(rin[s], ho);
    }
    // every load is issued; convert to FP32
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

    const BlockInfo bi = a.info[b];
    int bx, by, bz, gid;
    block_pos(bi, &bx, &by, &bz, &gid);
    const GeomInfo g = a.geom[gid];
    const int gx = bx * 8 + lx, gy = by * 8 + ly;
    const bool bnd = bx == 0 || by == 0 || bz == 0 || bx * 8 + 8 >= g.nx || by * 8 + 8 >= g.ny || bz * 8 + 8 >= g.nz;
    uint32_t dany = 0u;
#pragma unroll
    for (int s = 0; s < S; ++s) dany |= a.coef[s].dir;
    const bool dblk = bnd && dany != 0u;  // this block may hold Dirichlet voxels
    const uint32_t key = a.sround ? sr_key(*a.ctr + a.ctr_off, a.seed) : 0u;
    // ds_bpermute byte addresses: the row above / below (any lane; the face rows take
    // their halos instead)
    const int ym_addr = ((lane + 56) & 63) * 4, yp_addr = ((lane + 8) & 63) * 4;
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        const unsigned code = cd[z];
        const unsigned m = code & 63u;
        const int gz = bz * 8 + z;
        const unsigned onf = bnd ? ((gx == 0 ? 1u : 0u) | (gx == g.nx - 1 ? 2u : 0u) | (gy == 0 ? 4u : 0u) |
                                    (gy == g.ny - 1 ? 8u : 0u) | (gz == 0 ? 16u : 0u) | (gz == g.nz - 1 ? 32u : 0u))
                                 : 0u;
        const int nwall = __popc(~onf & ~m & 0x3fu);
        // halo sources of plane z: x faces at (u, v) = (y, z), y faces at (x, z)
        const int hx = (z * 8 + ly) * 4, hy = (z * 8 + lx) * 4;
        float res[S];
        const uint32_t h = a.sround ? sr_voxel(g, gx, gy, gz, key) : 0u;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const float cz = c[s][z];
            float xm = row_shift<1>(cz), xp = row_shift<-1>(cz);
            float ym = lane_read(ym_addr, cz), yp = lane_read(yp_addr, cz);
            const float hxm = lane_read(hx, side[0][s]), hxp = lane_read(hx, side[1][s]);
            const float hym = lane_read(hy, side[2][s]), hyp = lane_read(hy, side[3][s]);
            xm = lx == 0 ? hxm : xm;
            xp = lx == 7 ? hxp : xp;
            ym = ly == 0 ? hym : ym;
            yp = ly == 7 ? hyp : yp;
            const float dn = z == 0 ? zlo[s] : c[s][z > 0 ? z - 1 : 0];
            const float up = z == 7 ? zhi[s] : c[s][z < 7 ? z + 1 : 7];
            const float nbv[6] = {xm, xp, ym, yp, dn, up};
            float cen[S];
#pragma unroll
            for (int q = 0; q < S; ++q) cen[q] = c[q][z];
            const float dth = DTH ? fp32_dither(cz, sr_species(h, s)) : 0.0f;
            const float upd = rd_update<S, DTH>(cz, nbv, m, nwall, a.coef[s], cen, dth);
            res[s] = (dblk && (onf & a.coef[s].dir) != 0u) ? cz : upd;
        }
#pragma unroll
        for (int s = 0; s < S; ++s) Bt::st(rout[s], vo[z], res[s], a.sround != 0, sr_species(h, s));
    }
}

template <typename T, int S>
void launch_s(const StepArgs &a, int groups, hipStream_t st)
{
    if (sizeof(T) == 4 && a.sround) hipLaunchKernelGGL((k_step8l<T, S, true>), dim3(groups), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_step8l<T, S, false>), dim3(groups), dim3(256), 0, st, a);
}

template <typename T>
int launch_t(const StepArgs &a, hipStream_t st)
{
    int groups = (a.nb + 3) / 4;
    if (a.xcd_chunk > 0) groups = 8 * a.xcd_chunk;
    switch (a.S) {
    case 1: launch_s<T, 1>(a, groups, st); break;
    case 2: launch_s<T, 2>(a, groups, st); break;
    case 3: launch_s<T, 3>(a, groups, st); break;
    default: launch_s<T, 4>(a, groups, st); break;
    }
    return (int)hipGetLastError();
}

}  // namespace

// Step on the compact layout with lane-exchanged neighbours (a.cbase set, B = 8).
int rd_launch_step_lanes(int storage, const StepArgs &a, void *stream)
{
    if (a.nb <= 0) return 0;
    hipStream_t st = (hipStream_t)stream;
    if (storage == 0) return launch_t<float>(a, st);
    if (storage == 1) return launch_t<bf16_t>(a, st);
    return launch_t<_Float16>(a, st);
}
