// k_diff.hip -- FTCS step, balance and set-up kernels for inhomogeneous diffusion, for
// gfx950 (wave64).
//
// The diffusion coefficient of species s at a voxel is D_s * e, with e a per-slot FP32
// factor.  The flux through the face between voxels p and q uses the arithmetic mean
// of the two coefficients, and a face toward an inactive voxel (or the box edge)
// carries no flux: the neighbour takes the centre's value and coefficient (mirror
// rule).  This is the per-axis flux form of the inhomogeneous-diffusion functor in the
// paper's appendix "Code examples", with D(phi) from eq. inhomog_diffusion_coefficient
// (section "Level-set method for image-based geometry reconstruction").
//
// Kernels:
//   * k_step8e: B = 8, one wave per block, each lane walking a z-column; the fields
//     and the factor are staged plane by plane in LDS with their face halos.
//   * k_step_diff: any B, one thread per slot, neighbours read through the block
//     list.  Same arithmetic (rd_update_e) as k_step8e, so both give the same bits.
//   * k_set_diff: fills e from a dense array (values or the smooth D(phi)).
//   * k_reduce_diff: the balance terms, with the mean coefficient on Dirichlet faces.
// Like the homogeneous step this is HBM-bound: the factor adds 4 bytes per slot read.
// A volumetric sink on the near-surface band (code bit 7) rides along at no extra bytes.
#include "rd_device.h"
#include "rd_diff.h"

namespace {

__device__ __forceinline__ unsigned faces_on_box(const GeomInfo &g, int gx, int gy, int gz)
{
    return (gx == 0 ? 1u : 0u) | (gx == g.nx - 1 ? 2u : 0u) | (gy == 0 ? 4u : 0u) |
           (gy == g.ny - 1 ? 8u : 0u) | (gz == 0 ? 16u : 0u) | (gz == g.nz - 1 ? 32u : 0u);
}

__device__ __forceinline__ bool block_on_box(const GeomInfo &g, int bx, int by, int bz)
{
    return bx == 0 || by == 0 || bz == 0 || bx * 8 + 8 >= g.nx || by * 8 + 8 >= g.ny ||
           bz * 8 + 8 >= g.nz;
}

// Random word of a voxel for stochastic rounding (0 when rounding to nearest); the
// key and the per-voxel hash are those of the homogeneous step.
__device__ __forceinline__ uint32_t diff_key(const StepArgs &a)
{
    return a.sround ? sr_key(*a.ctr + a.ctr_off, a.seed) : 0u;
}

template <typename T>
__device__ __forceinline__ void diff_store(const StepArgs &a, T *cout, int s, int64_t idx, uint32_t h,
                                           float r)
{
    if (a.sround) rd_st_sr(cout, idx, r, sr_species(h, s));
    else rd_st(cout, idx, r);
}

// FTCS update of one free voxel with the factor:
//   lap = sum over active neighbours q (in -x,+x,-y,+y,-z,+z order) of
//         ((e_p + e_q) / 2) (c_q - c_p)
//   c'  = c + alpha lap - (beta + gamma n_wall + sk) c + sum_b K_b c_b
// alpha = D_s dt / dx^2, sk = dt k_s on band slots and 0 elsewhere.  The difference
// form keeps the error proportional to the local differences.
template <int S>
__device__ __forceinline__ float rd_update_e(float uc, const float nbv[6], const float ev[6], float ec,
                                             unsigned nbm, int nwall, const SpeciesCoef &k, float sk,
                                             const float *cen)
{
    float lap = 0.0f;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        const float w = 0.5f * (ec + ev[d]);
        lap = ((nbm >> d) & 1u) ? fmaf(w, nbv[d] - uc, lap) : lap;
    }
    float r = fmaf(k.alpha, lap, uc);
    const float loss = fmaf(k.gamma, (float)nwall, k.beta) + sk;
    r = fmaf(-loss, uc, r);
#pragma unroll
    for (int b = 0; b < S; ++b) r = fmaf(k.K[b], cen[b], r);
    return r;
}

// List index of the face neighbour slot of slot (lx, ly, lz) of block b in direction
// d, or -1 when the neighbour block is not stored.
template <int B>
__device__ __forceinline__ int64_t nbr_slot(const BlockInfo &bi, int b, int lx, int ly, int lz, int d)
{
    int x = lx, y = ly, z = lz, n = b;
    switch (d) {
    case 0: if (x > 0) --x; else { n = bi.nbr[0]; x = B - 1; } break;
    case 1: if (x < B - 1) ++x; else { n = bi.nbr[1]; x = 0; } break;
    case 2: if (y > 0) --y; else { n = bi.nbr[2]; y = B - 1; } break;
    case 3: if (y < B - 1) ++y; else { n = bi.nbr[3]; y = 0; } break;
    case 4: if (z > 0) --z; else { n = bi.nbr[4]; z = B - 1; } break;
    default: if (z < B - 1) ++z; else { n = bi.nbr[5]; z = 0; } break;
    }
    return n < 0 ? -1 : (int64_t)n * (B * B * B) + (z * B + y) * B + x;
}

// One thread per slot.  Inactive slots are not written (they hold 0 in both buffers).
template <typename T, int B, int S>
__global__ __launch_bounds__(256) void k_step_diff(DiffArgs d)
{
    constexpr int NS = B * B * B;
    const StepArgs &a = d.s;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)a.nb * NS) return;
    const unsigned code = a.code[i];
    if (!(code & 64u)) return;
    const int b = (int)(i / NS), slot = (int)(i % NS);
    const int lx = slot % B, ly = (slot / B) % B, lz = slot / (B * B);
    const BlockInfo bi = a.info[b];
    int bx, by, bz, gid;
    block_pos(bi, &bx, &by, &bz, &gid);
    const GeomInfo g = a.geom[gid];
    const int gx = bx * B + lx, gy = by * B + ly, gz = bz * B + lz;
    const unsigned onf = faces_on_box(g, gx, gy, gz);
    const unsigned m = code & 63u;
    const int nwall = __popc(~onf & ~m & 0x3fu);
    const T *cin = (const T *)a.cin;
    T *cout = (T *)a.cout;
    int64_t q[6];
    float ev[6];
#pragma unroll
    for (int dd = 0; dd < 6; ++dd) {
        const bool on = (m >> dd) & 1u;
        q[dd] = on ? nbr_slot<B>(bi, b, lx, ly, lz, dd) : i;
        ev[dd] = on ? d.e[q[dd]] : 0.0f;
    }
    const float ec = d.e[i];
    float cen[S];
#pragma unroll
    for (int s = 0; s < S; ++s) cen[s] = rd_ld(cin, s * a.sstride + i);
    const uint32_t h = a.sround ? sr_voxel(g, gx, gy, gz, diff_key(a)) : 0u;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        float nbv[6];
#pragma unroll
        for (int dd = 0; dd < 6; ++dd) nbv[dd] = ((m >> dd) & 1u) ? rd_ld(cin, s * a.sstride + q[dd]) : 0.0f;
        const float sk = (code & RD_CODE_BAND) ? d.sink[s] : 0.0f;
        const float upd = rd_update_e<S>(cen[s], nbv, ev, ec, m, nwall, a.coef[s], sk, cen);
        const bool isd = (onf & a.coef[s].dir) != 0u;
        diff_store(a, cout, s, s * a.sstride + i, h, isd ? cen[s] : upd);
    }
}

__device__ __forceinline__ int pix(int x, int y) { return (y + 1) * 10 + (x + 1); }

// B = 8 column form: four blocks per workgroup, one wave per block, lane (lx, ly)
// walking z.  Loads are predicated on the activity of the slot they read (inactive
// slots give 0); plane z of every species and of the factor goes to LDS with its
// four side halos, the z neighbours stay in registers.  Whole 128-byte sectors that
// hold an active voxel are stored.  XCH: the x faces of x-adjacent blocks of one
// workgroup are handed over through LDS instead of being read again.
template <typename T, int S, bool XCH>
__global__ __launch_bounds__(256) void k_step8e(DiffArgs d)
{
    __shared__ float tile[4][S + 1][100];  // species tiles, then the factor's
    __shared__ float xch[XCH ? 4 : 1][2][S + 1][64];  // x = 0 / x = 7 planes, [z * 8 + y]
    const StepArgs &a = d.s;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int grp = map_group(blockIdx.x, a.xcd_chunk);
    const int b = __builtin_amdgcn_readfirstlane(grp * 4 + wv);
    if (b >= a.nb) {  // past the end of the list (with XCH: after the one barrier)
        if (XCH) __syncthreads();
        return;
    }
    const T *cin = (const T *)a.cin;
    T *cout = (T *)a.cout;
    const int64_t base = (int64_t)b * 512;
    const int lx = lane & 7, ly = lane >> 3;
    // the block record whole and unconditionally: one scalar load instead of a load per
    // neighbour index behind the tests below
    const BlockInfo bi = a.info[b];
    const int32_t *nbr = bi.nbr;
    // x neighbours inside this workgroup (wave-uniform; only with XCH)
    const bool xm_in = XCH && wv > 0 && nbr[0] == b - 1;
    const bool xp_in = XCH && wv < 3 && nbr[1] == b + 1;
    const uint64_t *rec = a.mask + (int64_t)b * 16;
    uint64_t Wo[8], Wf[6];
#pragma unroll
    for (int z = 0; z < 8; ++z) Wo[z] = rec[z];
#pragma unroll
    for (int f = 0; f < 6; ++f) Wf[f] = rec[8 + f];

    typedef typename RawOf<T>::type R;
    R rc[S][8], rh[6][S];
    float ec[8], eh[6];
    unsigned cd[8];
#pragma unroll
    for (int z = 0; z < 8; ++z) {
#pragma unroll
        for (int s = 0; s < S; ++s) rc[s][z] = (R)0;
        ec[z] = 0.0f;
        cd[z] = 0u;
        if (lane_bit(Wo[z])) {
#pragma unroll
            for (int s = 0; s < S; ++s) rc[s][z] = ld_raw(cin, s * a.sstride + base + z * 64 + lane);
            ec[z] = d.e[base + z * 64 + lane];
            cd[z] = (unsigned)a.code[base + z * 64 + lane];
        }
    }
    // face halos: lane (u, v) = (lx, ly) reads the neighbour slot across face f at face
    // coordinates (u, v); a face bit is set only when the neighbour block exists
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
        const int64_t hb = (int64_t)(n >= 0 ? n : b) * 512 + ns;
#pragma unroll
        for (int s = 0; s < S; ++s) rh[f][s] = (R)0;
        eh[f] = 0.0f;
        if (lane_bit((f == 0 && xm_in) || (f == 1 && xp_in) ? 0ull : Wf[f])) {
#pragma unroll
            for (int s = 0; s < S; ++s) rh[f][s] = ld_raw(cin, s * a.sstride + hb);
            eh[f] = d.e[hb];
        }
    }
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
    // hand the x = 0 / x = 7 planes (species and factor) to the x neighbours of this
    // workgroup; inactive slots are 0 already, as a predicated halo load would give
    if (XCH) {
        if (lx == 0 || lx == 7) {
            const int side_ = lx == 7 ? 1 : 0;
#pragma unroll
            for (int z = 0; z < 8; ++z) {
#pragma unroll
                for (int s = 0; s < S; ++s) xch[wv][side_][s][z * 8 + ly] = c[s][z];
                xch[wv][side_][S][z * 8 + ly] = ec[z];
            }
        }
        __syncthreads();
        // face coordinates (u, v) = (lx, ly) of an x face are (y, z)
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (xm_in) side[0][s] = xch[wv - 1][1][s][ly * 8 + lx];
            if (xp_in) side[1][s] = xch[wv + 1][0][s][ly * 8 + lx];
        }
        if (xm_in) eh[0] = xch[wv - 1][1][S][ly * 8 + lx];
        if (xp_in) eh[1] = xch[wv + 1][0][S][ly * 8 + lx];
    }

    int bx, by, bz, gid;
    block_pos(bi, &bx, &by, &bz, &gid);
    const GeomInfo g = a.geom[gid];
    const int gx = bx * 8 + lx, gy = by * 8 + ly;
    const bool bnd = block_on_box(g, bx, by, bz);
    const uint32_t key = diff_key(a);
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        // plane z and its ring: the side halos of plane z are held by the lanes with
        // ly == z (face coordinate v = z, u = lx)
#pragma unroll
        for (int s = 0; s < S; ++s) {
            float *ts = tile[wv][s];
            ts[pix(lx, ly)] = c[s][z];
            if (ly == z) {
                ts[pix(-1, lx)] = side[0][s];
                ts[pix(8, lx)] = side[1][s];
                ts[pix(lx, -1)] = side[2][s];
                ts[pix(lx, 8)] = side[3][s];
            }
        }
        {
            float *te = tile[wv][S];
            te[pix(lx, ly)] = ec[z];
            if (ly == z) {
                te[pix(-1, lx)] = eh[0];
                te[pix(8, lx)] = eh[1];
                te[pix(lx, -1)] = eh[2];
                te[pix(lx, 8)] = eh[3];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        const int gz = bz * 8 + z;
        const unsigned code = cd[z];
        const unsigned m = code & 63u;
        const bool act = (code & 64u) != 0u;
        unsigned onf = 0u;
        if (bnd) onf = faces_on_box(g, gx, gy, gz);
        const int nwall = __popc(~onf & ~m & 0x3fu);
        const float *pe = &tile[wv][S][pix(lx, ly)];
        const float ev[6] = {pe[-1], pe[1], pe[-10], pe[10], z == 0 ? eh[4] : ec[z > 0 ? z - 1 : 0],
                             z == 7 ? eh[5] : ec[z < 7 ? z + 1 : 7]};
        float cen[S], res[S];
#pragma unroll
        for (int s = 0; s < S; ++s) cen[s] = c[s][z];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const float *p = &tile[wv][s][pix(lx, ly)];
            const float dn = z == 0 ? zlo[s] : c[s][z > 0 ? z - 1 : 0];
            const float up = z == 7 ? zhi[s] : c[s][z < 7 ? z + 1 : 7];
            const float nbv[6] = {p[-1], p[1], p[-10], p[10], dn, up};
            const float sk = (code & RD_CODE_BAND) ? d.sink[s] : 0.0f;
            const float upd = rd_update_e<S>(cen[s], nbv, ev, ec[z], m, nwall, a.coef[s], sk, cen);
            const bool isd = (onf & a.coef[s].dir) != 0u;
            res[s] = act ? (isd ? cen[s] : upd) : 0.0f;
        }
        // every lane has read plane z before any lane overwrites it with plane z + 1
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane_bit(sector_lanes<T>(Wo[z]))) {
            const uint32_t h = a.sround ? sr_voxel(g, gx, gy, gz, key) : 0u;
#pragma unroll
            for (int s = 0; s < S; ++s) diff_store(a, cout, s, s * a.sstride + base + z * 64 + lane, h, res[s]);
        }
    }
}

// e from a dense (nz, ny, nx) array, a grid-stride loop over the slots.  stats[0]
// counts active slots with a negative or non-finite value, stats[1] holds the largest
// valid value (FP32 bits; non-negative values order like their bit patterns).  The
// counts are reduced per workgroup first: one pair of atomics per workgroup.
template <int B>
__global__ __launch_bounds__(256) void k_set_diff(const BlockInfo *info, const uint8_t *code,
                                                  const GeomInfo *geom, int nb, const float *dense,
                                                  int mode, double d_min, double d_max, double g1,
                                                  double g2, float *e, uint32_t *stats)
{
    constexpr int NS = B * B * B;
    __shared__ uint32_t wbad[4], wmx[4];
    uint32_t nbad = 0u, mx = 0u;
    const int64_t n = (int64_t)nb * NS;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        float v = 0.0f;
        bool bad = false;
        if (code[i] & 64u) {
            const int b = (int)(i / NS), slot = (int)(i % NS);
            int bx, by, bz, gid;
            block_pos(info[b], &bx, &by, &bz, &gid);
            const GeomInfo g = geom[gid];
            const int gx = bx * B + slot % B, gy = by * B + (slot / B) % B, gz = bz * B + slot / (B * B);
            const float x = mode == 2 ? 1.0f : dense[voxel_id(g, gx, gy, gz)];
            v = mode != 1 ? x : (float)(d_min + d_max / (1.0 + exp(-(g1 + g2 * (double)x))));
            bad = !(v >= 0.0f) || !isfinite(v);
            if (!bad) mx = max(mx, __float_as_uint(v));
            nbad += bad ? 1u : 0u;
        }
        e[i] = bad ? 0.0f : v;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 64));
        nbad += (uint32_t)__shfl_xor((int)nbad, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        wbad[threadIdx.x >> 6] = nbad;
        wmx[threadIdx.x >> 6] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t tb = wbad[0] + wbad[1] + wbad[2] + wbad[3];
        const uint32_t tm = max(max(wmx[0], wmx[1]), max(wmx[2], wmx[3]));
        if (tb) atomicAdd(&stats[0], tb);
        if (tm) atomicMax(&stats[1], tm);
    }
}

// Balance terms with the factor.  B = 8: one block per workgroup, two slots per thread;
// B = 4: four blocks per workgroup, one slot per thread.  Lanes as in the homogeneous
// reduction: mass, inflow[6], uptake, reactions, non-finite count.  One row per
// workgroup: the wave sums in wave order.
template <typename T, int B>
__global__ __launch_bounds__(256) void k_reduce_diff(ReduceArgs a, const float *e, double ksink)
{
    using C = Cfg<B>;
    constexpr int NS = B * B * B;
    __shared__ double wsum[4][RD_NRED];
    double acc[RD_NRED];
#pragma unroll
    for (int l = 0; l < RD_NRED; ++l) acc[l] = 0.0;
    const int sub = threadIdx.x / C::TPB, lt = threadIdx.x % C::TPB;
    const int b = a.b0 + (int)blockIdx.x * C::BPW + sub;
    const T *c = (const T *)a.c;
    bool dblock = false;  // the block touches a Dirichlet face of the species (wave-uniform)
    if (b < a.b0 + a.nb) {
        const BlockInfo bi = a.info[b];
        int bx, by, bz, gid;
        block_pos(bi, &bx, &by, &bz, &gid);
        const GeomInfo g = a.geom[gid];
        const bool at[6] = {bx == 0, bx * B + B >= g.nx, by == 0, by * B + B >= g.ny, bz == 0,
                            bz * B + B >= g.nz};
        for (int f = 0; f < 6; ++f) dblock = dblock || (((a.dir >> f) & 1u) && at[f]);
        const double dx = a.dx, dx2 = dx * dx, dx3 = dx2 * dx;
        const T *cs = c + a.s * a.sstride;
        for (int k = 0; k < C::VPT; ++k) {
            const int slot = lt + k * C::TPB;
            const int64_t i = (int64_t)b * NS + slot;
            const unsigned code = a.code[i];
            if (!(code & 64u)) continue;
            const int lx = slot % B, ly = (slot / B) % B, lz = slot / (B * B);
            const int gx = bx * B + lx, gy = by * B + ly, gz = bz * B + lz;
            const unsigned nbm = code & 63u;
            const unsigned onf = faces_on_box(g, gx, gy, gz);
            const int nwall = __popc(~onf & ~nbm & 0x3fu);
            const float uf = rd_ld(cs, i);
            const double u = (double)uf;
            if (!isfinite(uf)) acc[9] += 1.0;
            if (onf & a.dir) {
                // first flagged face (in face order) this voxel lies on
                int fq = 0;
                for (int f = 5; f >= 0; --f)
                    if (((a.dir >> f) & 1u) && ((onf >> f) & 1u)) fq = f;
                const int ddx[6] = {-1, 1, 0, 0, 0, 0}, ddy[6] = {0, 0, -1, 1, 0, 0},
                          ddz[6] = {0, 0, 0, 0, -1, 1};
                const double eq = (double)e[i];
                double fin = 0.0;
                for (int d = 0; d < 6; ++d) {
                    if (!((nbm >> d) & 1u)) continue;
                    if (faces_on_box(g, gx + ddx[d], gy + ddy[d], gz + ddz[d]) & a.dir) continue;
                    const int64_t q = nbr_slot<B>(bi, b, lx, ly, lz, d);
                    const double dh = a.D * (0.5 * (eq + (double)e[q]));
                    fin += dh * (u - (double)rd_ld(cs, q)) * dx;
                }
                for (int f = 0; f < 6; ++f)
                    if (f == fq) acc[1 + f] += fin;
                continue;
            }
            acc[0] += u * dx3;
            acc[7] += a.kR * (double)nwall * u * dx2;
            if (code & RD_CODE_BAND) acc[7] += ksink * u * dx3;
            double re = -a.rate_out * u;
            for (int s2 = 0; s2 < a.S; ++s2)
                if (a.rate_in[s2] != 0.0) re += a.rate_in[s2] * (double)rd_ld(c, s2 * a.sstride + i);
            acc[8] += re * dx3;
        }
    }
    // wave sums of the lanes that can be nonzero (the others are 0 in every lane)
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    bool hasreact = a.rate_out != 0.0;
    for (int s2 = 0; s2 < a.S; ++s2) hasreact = hasreact || a.rate_in[s2] != 0.0;
#pragma unroll
    for (int l = 0; l < RD_NRED; ++l) {
        const bool need = l == 0 || l == 9 || (l <= 6 && dblock) || (l == 7 && (a.kR != 0.0 || ksink != 0.0)) ||
                          (l == 8 && hasreact);
        const double v = need ? wave_sum(acc[l]) : 0.0;
        if (lane == 0) wsum[wave][l] = v;
    }
    __syncthreads();
    if (threadIdx.x < RD_NRED) {
        const int l = threadIdx.x;
        a.partial[(int64_t)blockIdx.x * RD_NRED + l] = ((wsum[0][l] + wsum[1][l]) + wsum[2][l]) + wsum[3][l];
    }
}

// Flux through the plane i0 | i0 + 1 along axis with the mean face coefficient.  Rows as
// in k_reduce_diff; blocks that do not hold plane i0 return at once.
template <typename T, int B>
__global__ __launch_bounds__(256) void k_plane_flux_diff(const BlockInfo *info, const uint8_t *code, const T *c,
                                                         const float *e, int nb, int axis, int i0, double D,
                                                         double dx, double *partial)
{
    using C = Cfg<B>;
    constexpr int NS = B * B * B;
    __shared__ double wsum[4];
    const int sub = threadIdx.x / C::TPB, lt = threadIdx.x % C::TPB;
    const int b = blockIdx.x * C::BPW + sub;
    double acc = 0.0;
    if (b < nb) {
        const BlockInfo bi = info[b];
        int bx, by, bz, gid;
        block_pos(bi, &bx, &by, &bz, &gid);
        const int o = (axis == 0 ? bx : axis == 1 ? by : bz) * B;
        if (i0 >= o && i0 < o + B) {
            const int l0 = i0 - o;
            for (int k = 0; k < C::VPT; ++k) {
                const int slot = lt + k * C::TPB;
                const int lx = slot % B, ly = (slot / B) % B, lz = slot / (B * B);
                if ((axis == 0 ? lx : axis == 1 ? ly : lz) != l0) continue;
                const int64_t i = (int64_t)b * NS + slot;
                const unsigned cd = code[i];
                if (!(cd & 64u) || !((cd >> (2 * axis + 1)) & 1u)) continue;
                const int64_t q = nbr_slot<B>(bi, b, lx, ly, lz, 2 * axis + 1);
                const double w = 0.5 * ((double)e[i] + (double)e[q]);
                acc += D * w * ((double)rd_ld(c, i) - (double)rd_ld(c, q)) * dx;
            }
        }
    }
    const double v = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
}

// Band marking, a grid-stride loop over the slots; one atomic per workgroup.
template <int B>
__global__ __launch_bounds__(256) void k_set_band(const BlockInfo *info, uint8_t *code, const GeomInfo *geom,
                                                  int nb, const float *phi, double band, uint32_t *count)
{
    constexpr int NS = B * B * B;
    __shared__ uint32_t wn[4];
    uint32_t cnt = 0u;
    const int64_t n = (int64_t)nb * NS;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const unsigned c = code[i];
        if (c & 64u) {
            const int b = (int)(i / NS), slot = (int)(i % NS);
            int bx, by, bz, gid;
            block_pos(info[b], &bx, &by, &bz, &gid);
            const GeomInfo g = geom[gid];
            const int gx = bx * B + slot % B, gy = by * B + (slot / B) % B, gz = bz * B + slot / (B * B);
            const bool in = (double)phi[voxel_id(g, gx, gy, gz)] < band;
            code[i] = (uint8_t)((c & 0x7fu) | (in ? RD_CODE_BAND : 0u));
            cnt += in ? 1u : 0u;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) cnt += (uint32_t)__shfl_xor((int)cnt, o, 64);
    if ((threadIdx.x & 63) == 0) wn[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t t = wn[0] + wn[1] + wn[2] + wn[3];
        if (t) atomicAdd(count, t);
    }
}

template <typename T, int B, int S>
void launch_diff_s(const DiffArgs &a, int column, hipStream_t st)
{
    if (B == 8 && column) {
        int groups = (a.s.nb + 3) / 4;
        if (a.s.xcd_chunk > 0) groups = 8 * a.s.xcd_chunk;
        if (column == 2) hipLaunchKernelGGL((k_step8e<T, S, true>), dim3(groups), dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_step8e<T, S, false>), dim3(groups), dim3(256), 0, st, a);
    } else {
        const int64_t n = (int64_t)a.s.nb * B * B * B;
        hipLaunchKernelGGL((k_step_diff<T, B, S>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a);
    }
}

template <typename T, int B>
void launch_diff_t(const DiffArgs &a, int column, hipStream_t st)
{
    switch (a.s.S) {
    case 1: launch_diff_s<T, B, 1>(a, column, st); break;
    case 2: launch_diff_s<T, B, 2>(a, column, st); break;
    case 3: launch_diff_s<T, B, 3>(a, column, st); break;
    default: launch_diff_s<T, B, 4>(a, column, st); break;
    }
}

template <typename T>
void launch_diff_b(int B, const DiffArgs &a, int column, hipStream_t st)
{
    if (B == 8) launch_diff_t<T, 8>(a, column, st);
    else launch_diff_t<T, 4>(a, column, st);
}

template <typename T>
void launch_reduce_b(int B, const ReduceArgs &a, const float *e, double ksink, hipStream_t st)
{
    const dim3 grid((unsigned)rd_diff_reduce_rows(B, a.nb));
    if (B == 8) hipLaunchKernelGGL((k_reduce_diff<T, 8>), grid, dim3(256), 0, st, a, e, ksink);
    else hipLaunchKernelGGL((k_reduce_diff<T, 4>), grid, dim3(256), 0, st, a, e, ksink);
}

}  // namespace

int rd_launch_step_diff(int storage, int B, const DiffArgs &a, int column, void *stream)
{
    if (a.s.nb <= 0) return 0;
    hipStream_t st = (hipStream_t)stream;
    if (storage == 0) launch_diff_b<float>(B, a, column, st);
    else if (storage == 1) launch_diff_b<bf16_t>(B, a, column, st);
    else launch_diff_b<_Float16>(B, a, column, st);
    return (int)hipGetLastError();
}

int rd_launch_set_diff(int B, const BlockInfo *info, const uint8_t *code, const GeomInfo *geom, int nb,
                       const float *dense, int mode, double d_min, double d_max, double g1, double g2,
                       float *e, uint32_t *stats, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    int rc = rd_launch_fill_u32(stats, 0u, 2, stream);
    if (rc != 0 || nb <= 0) return rc;
    const int64_t n = (int64_t)nb * B * B * B;
    const int64_t blocks = (n + 255) / 256;
    const dim3 grid((unsigned)(blocks < 4096 ? blocks : 4096));  // grid-stride
    if (B == 8)
        hipLaunchKernelGGL((k_set_diff<8>), grid, dim3(256), 0, st, info, code, geom, nb, dense, mode, d_min,
                           d_max, g1, g2, e, stats);
    else
        hipLaunchKernelGGL((k_set_diff<4>), grid, dim3(256), 0, st, info, code, geom, nb, dense, mode, d_min,
                           d_max, g1, g2, e, stats);
    return (int)hipGetLastError();
}

int rd_diff_reduce_rows(int B, int nb) { return B == 8 ? nb : (nb + 3) / 4; }

int rd_launch_reduce_diff(int storage, int B, const ReduceArgs &a, const float *e, double ksink, void *stream)
{
    if (a.nb <= 0) return 0;
    hipStream_t st = (hipStream_t)stream;
    if (storage == 0) launch_reduce_b<float>(B, a, e, ksink, st);
    else if (storage == 1) launch_reduce_b<bf16_t>(B, a, e, ksink, st);
    else launch_reduce_b<_Float16>(B, a, e, ksink, st);
    return (int)hipGetLastError();
}

int rd_launch_set_band(int B, const BlockInfo *info, uint8_t *code, const GeomInfo *geom, int nb, const float *phi,
                       double band, uint32_t *count, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    int rc = rd_launch_fill_u32(count, 0u, 1, stream);
    if (rc != 0 || nb <= 0) return rc;
    const int64_t n = (int64_t)nb * B * B * B;
    const int64_t blocks = (n + 255) / 256;
    const dim3 grid((unsigned)(blocks < 4096 ? blocks : 4096));  // grid-stride
    if (B == 8)
        hipLaunchKernelGGL((k_set_band<8>), grid, dim3(256), 0, st, info, code, geom, nb, phi, band, count);
    else
        hipLaunchKernelGGL((k_set_band<4>), grid, dim3(256), 0, st, info, code, geom, nb, phi, band, count);
    return (int)hipGetLastError();
}

int rd_launch_plane_flux_diff(int storage, int B, const BlockInfo *info, const uint8_t *code, const void *c,
                              const float *e, int nb, int axis, int i0, double D, double dx, double *partial,
                              void *stream)
{
    if (nb <= 0) return 0;
    hipStream_t st = (hipStream_t)stream;
    const dim3 grid((unsigned)rd_diff_reduce_rows(B, nb));
#define RD_PF(T, BB) \
    hipLaunchKernelGGL((k_plane_flux_diff<T, BB>), grid, dim3(256), 0, st, info, code, (const T *)c, e, nb, axis, i0, \
                       D, dx, partial)
    if (B == 8) {
        if (storage == 0) RD_PF(float, 8);
        else if (storage == 1) RD_PF(bf16_t, 8);
        else RD_PF(_Float16, 8);
    } else {
        if (storage == 0) RD_PF(float, 4);
        else if (storage == 1) RD_PF(bf16_t, 4);
        else RD_PF(_Float16, 4);
    }
#undef RD_PF
    return (int)hipGetLastError();
}
