// k_solve.hip -- conjugate gradients for the steady state of pure diffusion on the
// sparse block grid, for one geometry or a batch of concatenated geometries.
//
// Problem (the t -> infinity limit of the FTCS step with the same mirror rule):
// on every free voxel p (active, not Dirichlet)
//     (A x)_p = sum over active face neighbours q of (x_p - x_q) = b_p,
// b_p = sum of the Dirichlet neighbours' held values.  A is the graph Laplacian of
// the free voxels with Dirichlet contacts on the diagonal: symmetric positive
// semi-definite, so plain CG applies.  Vectors live in the storage type T with FP32
// arithmetic; every dot product is an FP64 per-block partial summed per geometry in
// a fixed order.  Tortuosity follows from the steady flux (eq. tortuosity).
#include <algorithm>

#include "rd_device.h"
#include "rd_solve.h"

namespace {

// Per-block sum of two FP64 values over the block's voxels, written to part[b*2 + k].
// B = 8: one block spans the 4 waves; B = 4: one block is one wave.
template <int B>
__device__ __forceinline__ void block_sum2(double v0, double v1, double *part, int b, bool valid)
{
    __shared__ double sh[4][2];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    v0 = wave_sum(v0);
    v1 = wave_sum(v1);
    if constexpr (B == 8) {
        if (lane == 0) {
            sh[wave][0] = v0;
            sh[wave][1] = v1;
        }
        __syncthreads();
        if (threadIdx.x == 0 && valid) {
            part[(int64_t)b * 2 + 0] = ((sh[0][0] + sh[1][0]) + sh[2][0]) + sh[3][0];
            part[(int64_t)b * 2 + 1] = ((sh[0][1] + sh[1][1]) + sh[2][1]) + sh[3][1];
        }
    } else {
        if (lane == 0 && valid) {
            part[(int64_t)b * 2 + 0] = v0;
            part[(int64_t)b * 2 + 1] = v1;
        }
    }
}

struct VoxCtx {
    bool act, fr;
    unsigned nbm;     // active neighbours
    unsigned dirnb;   // active neighbours that are Dirichlet voxels
    int gx, gy, gz;
};

template <int B>
__device__ __forceinline__ VoxCtx vox_ctx(const uint64_t *rec, const BlockInfo &bi, const GeomInfo &g,
                                          uint32_t dir, int slot)
{
    VoxCtx v;
    int bx, by, bz, gid;
    block_pos(bi, &bx, &by, &bz, &gid);
    const int lx = slot % B, ly = (slot / B) % B, lz = slot / (B * B);
    v.gx = bx * B + lx;
    v.gy = by * B + ly;
    v.gz = bz * B + lz;
    v.act = own_bit<B>(rec, slot);
    int nw = 0;
    v.nbm = v.act ? nb_bits<B>(rec, lx, ly, lz, v.gx, v.gy, v.gz, g.nx, g.ny, g.nz, &nw) : 0u;
    v.fr = v.act && !on_dirichlet(dir, v.gx, v.gy, v.gz, g.nx, g.ny, g.nz);
    const int ddx[6] = {-1, 1, 0, 0, 0, 0}, ddy[6] = {0, 0, -1, 1, 0, 0}, ddz[6] = {0, 0, 0, 0, -1, 1};
    unsigned d = 0;
#pragma unroll
    for (int k = 0; k < 6; ++k)
        if (((v.nbm >> k) & 1u) &&
            on_dirichlet(dir, v.gx + ddx[k], v.gy + ddy[k], v.gz + ddz[k], g.nx, g.ny, g.nz))
            d |= 1u << k;
    v.dirnb = d;
    return v;
}

// sum over active neighbours of (t_q - t_p), order -x,+x,-y,+y,-z,+z
template <int B>
__device__ __forceinline__ float lap_at(const float *ts, int t, unsigned nbm)
{
    using K = Blk<B>;
    const float uc = ts[t];
    const float nbv[6] = {ts[t - 1], ts[t + 1], ts[t - K::E], ts[t + K::E], ts[t - K::E * K::E],
                          ts[t + K::E * K::E]};
    float lap = 0.0f;
#pragma unroll
    for (int d = 0; d < 6; ++d) lap = ((nbm >> d) & 1u) ? lap + (nbv[d] - uc) : lap;
    return lap;
}

// (A p)_p on a free voxel of an 8^3 column kernel: the sum over active neighbours q of
// (p_p - p_q), in the order -x, +x, -y, +y, -z, +z; q points at p_p in the one-plane
// LDS tile, dn / up are the -z / +z values, `code` holds the active-neighbour bits.  0
// elsewhere.  The difference form keeps the rounding error proportional to the local
// differences, not to |p|: CG corrections are smooth fields far larger than their
// right-hand side, where n p_p - sum p_q would cancel catastrophically in FP32.
__device__ __forceinline__ float cg_ap8(const float *q, float dn, float up, float pc, unsigned code,
                                        bool fr)
{
    const float nv[6] = {q[-1], q[1], q[-10], q[10], dn, up};
    float ap = 0.0f;
#pragma unroll
    for (int d = 0; d < 6; ++d) ap = ((code >> d) & 1u) ? ap + (pc - nv[d]) : ap;
    return fr ? ap : 0.0f;
}

// Block-Jacobi preconditioner of the 8^3 column kernels: z = M^-1 r with
//   z_0 = V r,  z_{j+1} = V (r + N z_j),  j < steps - 1,
// V = diag(1 / n_p) over the free voxels (n_p: active neighbours of p, Dirichlet ones
// included, i.e. the diagonal of A) and N the adjacency of the free voxels of the same
// block: Jacobi steps on the block's own equations with every neighbour outside the
// block taken as 0.  M^-1 = sum_j (V N)^j V = V^1/2 (sum_j (V^1/2 N V^1/2)^j) V^1/2 is
// symmetric, and positive definite on every block component that has a neighbour
// outside it or a Dirichlet contact (there |eigenvalue of V^1/2 N V^1/2| < 1); an even
// step count keeps it well conditioned.  The same linear map in every kernel (same
// operations, same order), so CG sees one fixed preconditioner.
// ts: the wave's 10 x 10 LDS tile with a zero ring; rk: the lane's residual per plane
// (0 off free voxels); vk: 1 / n_p on free voxels, 0 elsewhere (z stays 0 there).
__device__ __forceinline__ void cg_jacobi8(float *ts, int lx, int ly, const float rk[8], const float vk[8],
                                           int steps, float zk[8])
{
#pragma unroll
    for (int k = 0; k < 8; ++k) zk[k] = rk[k] * vk[k];
    for (int j = 1; j < steps; ++j) {
        float zn[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            ts[(ly + 1) * 10 + (lx + 1)] = zk[k];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const float *q = &ts[(ly + 1) * 10 + (lx + 1)];
            const float dn = k > 0 ? zk[k > 0 ? k - 1 : 0] : 0.0f;
            const float up = k < 7 ? zk[k < 7 ? k + 1 : 7] : 0.0f;
            const float sum = ((q[-1] + q[1]) + (q[-10] + q[10])) + (dn + up);
            zn[k] = (rk[k] + sum) * vk[k];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) zk[k] = zn[k];
    }
}

// the ring of a wave's 10 x 10 tile set to 0 (lanes of the first row write it)
__device__ __forceinline__ void tile_ring_zero(float *ts, int lx, int ly)
{
    if (ly == 0) {
        ts[(lx + 1) * 10 + 0] = 0.0f;
        ts[(lx + 1) * 10 + 9] = 0.0f;
        ts[0 * 10 + (lx + 1)] = 0.0f;
        ts[9 * 10 + (lx + 1)] = 0.0f;
    }
}

// 1 / (active neighbours) of a free voxel from its code (0 for a voxel without any)
__device__ __forceinline__ float cg_inv_count(unsigned code)
{
    const unsigned n = (unsigned)__popc(code & 63u);
    return n ? __builtin_amdgcn_rcpf((float)n) : 0.0f;
}

template <int B>
__device__ __forceinline__ bool geom_live(const CgArgs &a, int gid)
{
    return a.scal[gid * CG_NSCAL + CG_DONE] == 0.0;
}

// Ap = A p on live geometries, partial (p.Ap, 0)
template <typename T, int B>
__global__ __launch_bounds__(256) void k_cg_matvec(CgArgs a)
{
    using K = Blk<B>;
    using C = Cfg<B>;
    __shared__ float tile[C::BPW][1][K::TL];
    __shared__ uint64_t srec[C::BPW][K::MW];
    const int sub = threadIdx.x / C::TPB, lt = threadIdx.x % C::TPB;
    const int b = blockIdx.x * C::BPW + sub;
    bool valid = b < a.nb;
    BlockInfo bi = {};
    if (valid) {
        bi = a.info[b];
        int bx, by, bz, gid;
        block_pos(bi, &bx, &by, &bz, &gid);
        valid = geom_live<B>(a, gid);
    }
    if (valid && lt < K::MW) srec[sub][lt] = a.mask[(int64_t)b * K::MW + lt];
    stage_tile<T, B>(tile[sub], (const T *)a.p, 0, 1, b, bi, lt, valid);
    __syncthreads();
    double pap = 0.0;
    if (valid) {
        int bx, by, bz, gid;
        block_pos(bi, &bx, &by, &bz, &gid);
        const GeomInfo g = a.geom[gid];
        for (int k = 0; k < C::VPT; ++k) {
            const int slot = lt + k * C::TPB;
            const VoxCtx v = vox_ctx<B>(srec[sub], bi, g, a.dir, slot);
            const int lx = slot % B, ly = (slot / B) % B, lz = slot / (B * B);
            const int t = K::tidx(lx, ly, lz);
            float ap = 0.0f;
            if (v.fr) {
                ap = -lap_at<B>(tile[sub][0], t, v.nbm);
                pap += (double)tile[sub][0][t] * (double)ap;
            }
            rd_st_keep((T *)a.ap, (int64_t)b * K::NS + slot, ap);
        }
    }
    block_sum2<B>(pap, 0.0, a.partial, b, b < a.nb);
}

// Ap = A p for 8^3 blocks in the column form of the step kernel: one wave per block,
// four blocks per workgroup, lane (lx, ly) walking its z-column, +-x / +-y
// neighbours through a one-plane LDS tile, every load predicated on the activity of
// the voxel it reads.  p is 0 on inactive and Dirichlet voxels (the residual and the
// p update never give them another value), so on a free voxel
//   (A p)_p = n_active * p_p - (((((p_-x + p_+x) + p_-y) + p_+y) + p_-z) + p_+z),
// and Ap = 0 elsewhere.  Partial (p.Ap, 0) per block in FP64.
// The p update of the previous iteration is applied on the fly, to the block and to
// its halos: p_new = fma(beta, p, r) from the stored r and p (the p update's own
// operation, rounded to the storage type), stored into p2 (the caller swaps the
// buffers: neighbouring waves still read the old p); Ap = A p_new.  p_new is 0 where
// r and p are (inactive and Dirichlet voxels).  Ap itself is not stored: the update
// kernel (k_cg_update8) recomputes it from p_new with the same arithmetic (cg_ap8),
// which moves fewer bytes than writing and reading it back.

// The four blocks of a workgroup are consecutive list entries; x-adjacent ones hand each
// other their x = 0 / x = 7 planes through LDS (one barrier) instead of loading the
// neighbour's strided x face, which touches every line of the neighbour block.  Every
// wave reaches the barrier, also those past the list or of converged geometries.
template <typename T>
__global__ __launch_bounds__(256) void k_cg_matvec8(CgArgs a)
{
    __shared__ float tile[4][100];
    __shared__ float xch[4][2][64];  // x = 0 / x = 7 planes of each wave's p_new, [z * 8 + y]
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int b = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + wv);
    if (b >= a.nb) {
        __syncthreads();
        return;
    }
    const BlockInfo bi = a.info[b];
    int bx, by, bz, gid;
    block_pos(bi, &bx, &by, &bz, &gid);
    if (!geom_live<8>(a, gid)) {
        if (lane == 0) {
            a.partial[(int64_t)b * 2 + 0] = 0.0;
            a.partial[(int64_t)b * 2 + 1] = 0.0;
        }
        __syncthreads();
        return;
    }
    // x neighbours inside this workgroup (same geometry, so live as well)
    const bool xm_in = wv > 0 && bi.nbr[0] == b - 1;
    const bool xp_in = wv < 3 && bi.nbr[1] == b + 1;
    const T *pv = (const T *)a.p;
    const int64_t base = (int64_t)b * 512;
    const int lx = lane & 7, ly = lane >> 3;
    const uint64_t *rec = a.mask + (int64_t)b * 16;
    uint64_t Wo[8], Wf[6];
#pragma unroll
    for (int z = 0; z < 8; ++z) Wo[z] = rec[z];
#pragma unroll
    for (int f = 0; f < 6; ++f) Wf[f] = rec[8 + f];
    typedef typename RawOf<T>::type R;
    const T *rv = (const T *)(a.prec > 0 ? a.z : a.r);  // p_new = z + beta p
    R rc[8], rh[6], qc[8], qh[6];  // p and z raw words
    unsigned cd[8];
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        const bool act = (Wo[z] >> lane) & 1ull;
        rc[z] = ld_raw(pv, base + z * 64 + lane, act);
        qc[z] = ld_raw(rv, base + z * 64 + lane, act);
        cd[z] = act ? (unsigned)a.code[base + z * 64 + lane] : 0u;
    }
    // face halos: lane (u, v) = (lx, ly) reads the neighbour slot across face f
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        int ns;
        switch (f) {
        case 0: ns = (ly * 8 + lx) * 8 + 7; break;
        case 1: ns = (ly * 8 + lx) * 8 + 0; break;
        case 2: ns = (ly * 8 + 7) * 8 + lx; break;
        case 3: ns = (ly * 8 + 0) * 8 + lx; break;
        case 4: ns = (7 * 8 + ly) * 8 + lx; break;
        default: ns = (0 * 8 + ly) * 8 + lx; break;
        }
        const int n = bi.nbr[f];
        const bool e = ((Wf[f] >> lane) & 1ull) && !(f == 0 && xm_in) && !(f == 1 && xp_in);
        rh[f] = ld_raw(pv, (int64_t)(n >= 0 ? n : b) * 512 + ns, e);
        qh[f] = ld_raw(rv, (int64_t)(n >= 0 ? n : b) * 512 + ns, e);
    }
    const float beta = (float)a.scal[gid * CG_NSCAL + CG_BETA];
    // the updated p, as the p update would have stored it
    auto pval = [&](R praw, R rraw) {
        return rd_round<T>(fmaf(beta, from_raw<T>(praw), from_raw<T>(rraw)));
    };
    float c[8], side[4];
#pragma unroll
    for (int z = 0; z < 8; ++z) c[z] = pval(rc[z], qc[z]);
#pragma unroll
    for (int f = 0; f < 4; ++f) side[f] = pval(rh[f], qh[f]);
    const float zlo = pval(rh[4], qh[4]), zhi = pval(rh[5], qh[5]);
    // the neighbour's p_new on its face: the value this wave would form from the halos
    if (lx == 0 || lx == 7) {
#pragma unroll
        for (int z = 0; z < 8; ++z) xch[wv][lx == 7 ? 1 : 0][z * 8 + ly] = c[z];
    }
    __syncthreads();
    if (xm_in) side[0] = xch[wv - 1][1][ly * 8 + lx];
    if (xp_in) side[1] = xch[wv + 1][0][ly * 8 + lx];

    const GeomInfo g = a.geom[gid];
    const int gx = bx * 8 + lx, gy = by * 8 + ly;
    const bool bnd = bx == 0 || by == 0 || bz == 0 || bx * 8 + 8 >= g.nx || by * 8 + 8 >= g.ny ||
                     bz * 8 + 8 >= g.nz;
    float *ts = tile[wv];
    double pap = 0.0;
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        ts[(ly + 1) * 10 + (lx + 1)] = c[z];
        if (ly == z) {  // side halos of plane z (face coordinate v = z)
            ts[(lx + 1) * 10 + 0] = side[0];
            ts[(lx + 1) * 10 + 9] = side[1];
            ts[0 * 10 + (lx + 1)] = side[2];
            ts[9 * 10 + (lx + 1)] = side[3];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const unsigned code = cd[z];
        unsigned onf = 0u;
        if (bnd)
            onf = (gx == 0 ? 1u : 0u) | (gx == g.nx - 1 ? 2u : 0u) | (gy == 0 ? 4u : 0u) |
                  (gy == g.ny - 1 ? 8u : 0u) | (bz * 8 + z == 0 ? 16u : 0u) |
                  (bz * 8 + z == g.nz - 1 ? 32u : 0u);
        const bool fr = (code & 64u) != 0u && (onf & a.dir) == 0u;
        const float *q = &ts[(ly + 1) * 10 + (lx + 1)];
        const float dn = z == 0 ? zlo : c[z > 0 ? z - 1 : 0];
        const float up = z == 7 ? zhi : c[z < 7 ? z + 1 : 7];
        const float ap = cg_ap8(q, dn, up, c[z], code, fr);
        if (fr) pap += (double)c[z] * (double)ap;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // whole sectors only (p is read on active voxels and as predicated halos)
        if (sector_active<T>(Wo[z], lane)) rd_st_keep((T *)a.p2, base + z * 64 + lane, c[z]);
    }
    pap = wave_sum(pap);
    if (lane == 0) {
        a.partial[(int64_t)b * 2 + 0] = pap;
        a.partial[(int64_t)b * 2 + 1] = 0.0;
    }
}

// x += alpha p, r -= alpha A p on free voxels of live geometries, for 8^3 blocks in the
// column form of k_cg_matvec8, which does not store A p: it is recomputed here from p
// and its face halos with the matvec's arithmetic (cg_ap8), so it equals the A p of
// the p.Ap partial bit for bit.  Whole sectors are stored: inactive slots keep 0 and
// Dirichlet voxels their values.  Partial (r.r, 0) per block, of r as stored.
// (Unlike the matvec, this kernel loads the x faces of one vector only; handing them
// over through LDS measured slower here: 499 against 486 us per call on a 512^3 foam.)
// PREC: the block's new residual, as stored, is preconditioned in place (cg_jacobi8:
// the whole block is in the wave's registers) and z = M^-1 r stored; partial (r.z, r.r).
// Without it the partial is (r.r, r.r).
template <typename T, bool X64, bool PREC>
__global__ __launch_bounds__(256) void k_cg_update8(CgArgs a)
{
    __shared__ float tile[4][100];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int b = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + wv);
    if (b >= a.nb) return;
    const BlockInfo bi = a.info[b];
    int bx, by, bz, gid;
    block_pos(bi, &bx, &by, &bz, &gid);
    if (!geom_live<8>(a, gid)) {
        if (lane == 0) {
            a.partial[(int64_t)b * 2 + 0] = 0.0;
            a.partial[(int64_t)b * 2 + 1] = 0.0;
        }
        return;
    }
    const T *pv = (const T *)a.p;
    T *xv = (T *)a.x;
    T *rv = (T *)a.r;
    const int64_t base = (int64_t)b * 512;
    const int lx = lane & 7, ly = lane >> 3;
    const uint64_t *rec = a.mask + (int64_t)b * 16;
    uint64_t Wo[8], Wf[6];
#pragma unroll
    for (int z = 0; z < 8; ++z) Wo[z] = rec[z];
#pragma unroll
    for (int f = 0; f < 6; ++f) Wf[f] = rec[8 + f];
    typedef typename RawOf<T>::type R;
    R pc[8], ph[6], xc[8], rc[8];
    double xd[8];
    unsigned cd[8];
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        const bool act = (Wo[z] >> lane) & 1ull;
        pc[z] = ld_raw(pv, base + z * 64 + lane, act);
        if (X64) xd[z] = act ? a.x64[base + z * 64 + lane] : 0.0;
        else xc[z] = ld_raw((const T *)xv, base + z * 64 + lane, act);
        rc[z] = ld_raw((const T *)rv, base + z * 64 + lane, act);
        cd[z] = act ? (unsigned)a.code[base + z * 64 + lane] : 0u;
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        int ns;
        switch (f) {
        case 0: ns = (ly * 8 + lx) * 8 + 7; break;
        case 1: ns = (ly * 8 + lx) * 8 + 0; break;
        case 2: ns = (ly * 8 + 7) * 8 + lx; break;
        case 3: ns = (ly * 8 + 0) * 8 + lx; break;
        case 4: ns = (7 * 8 + ly) * 8 + lx; break;
        default: ns = (0 * 8 + ly) * 8 + lx; break;
        }
        const int n = bi.nbr[f];
        const bool e = (Wf[f] >> lane) & 1ull;
        ph[f] = ld_raw(pv, (int64_t)(n >= 0 ? n : b) * 512 + ns, e);
    }
    const double alpha_d = a.scal[gid * CG_NSCAL + CG_ALPHA];
    const float alpha = (float)alpha_d;
    const double alpha_x = X64 ? alpha_d / a.scal[gid * CG_NSCAL + CG_SIGMA] : 0.0;  // p holds sigma p
    float c[8], side[4];
#pragma unroll
    for (int z = 0; z < 8; ++z) c[z] = from_raw<T>(pc[z]);
#pragma unroll
    for (int f = 0; f < 4; ++f) side[f] = from_raw<T>(ph[f]);
    const float zlo = from_raw<T>(ph[4]), zhi = from_raw<T>(ph[5]);

    const GeomInfo g = a.geom[gid];
    const int gx = bx * 8 + lx, gy = by * 8 + ly;
    const bool bnd = bx == 0 || by == 0 || bz == 0 || bx * 8 + 8 >= g.nx || by * 8 + 8 >= g.ny ||
                     bz * 8 + 8 >= g.nz;
    float *ts = tile[wv];
    double rr = 0.0;
    float rk[8], vk[8];  // PREC: the stored new residual and 1 / n_p (0 off free voxels)
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        ts[(ly + 1) * 10 + (lx + 1)] = c[z];
        if (ly == z) {
            ts[(lx + 1) * 10 + 0] = side[0];
            ts[(lx + 1) * 10 + 9] = side[1];
            ts[0 * 10 + (lx + 1)] = side[2];
            ts[9 * 10 + (lx + 1)] = side[3];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const unsigned code = cd[z];
        unsigned onf = 0u;
        if (bnd)
            onf = (gx == 0 ? 1u : 0u) | (gx == g.nx - 1 ? 2u : 0u) | (gy == 0 ? 4u : 0u) |
                  (gy == g.ny - 1 ? 8u : 0u) | (bz * 8 + z == 0 ? 16u : 0u) |
                  (bz * 8 + z == g.nz - 1 ? 32u : 0u);
        const bool fr = (code & 64u) != 0u && (onf & a.dir) == 0u;
        const float *q = &ts[(ly + 1) * 10 + (lx + 1)];
        const float dn = z == 0 ? zlo : c[z > 0 ? z - 1 : 0];
        const float up = z == 7 ? zhi : c[z < 7 ? z + 1 : 7];
        const float ap = cg_ap8(q, dn, up, c[z], code, fr);
        const float r0 = from_raw<T>(rc[z]);
        const float rn = fr ? fmaf(-alpha, ap, r0) : r0;
        float xn = 0.0f;
        double xdn = 0.0;
        if (X64) xdn = fr ? fma(alpha_x, (double)c[z], xd[z]) : xd[z];
        else xn = fr ? fmaf(alpha, c[z], from_raw<T>(xc[z])) : from_raw<T>(xc[z]);
        const float rs = rd_round<T>(rn);  // as stored
        if (fr) rr += (double)rs * (double)rs;
        if (PREC) {
            rk[z] = fr ? rs : 0.0f;
            vk[z] = fr ? cg_inv_count(code) : 0.0f;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (sector_active<T>(Wo[z], lane)) {
            if (!X64) rd_st_keep(xv, base + z * 64 + lane, xn);
            rd_st_keep(rv, base + z * 64 + lane, rn);
        }
        if (X64 && sector_active<double>(Wo[z], lane)) a.x64[base + z * 64 + lane] = xdn;
    }
    double rz = rr;
    if (PREC) {
        tile_ring_zero(ts, lx, ly);
        float zk[8];
        cg_jacobi8(ts, lx, ly, rk, vk, a.prec, zk);
        rz = 0.0;
#pragma unroll
        for (int z = 0; z < 8; ++z) {
            const float zs = rd_round<T>(zk[z]);  // as stored
            rz += (double)rk[z] * (double)zs;
            if (sector_active<T>(Wo[z], lane)) rd_st_keep((T *)a.z, base + z * 64 + lane, zk[z]);
        }
        rz = wave_sum(rz);
    }
    rr = wave_sum(rr);
    if (lane == 0) {
        a.partial[(int64_t)b * 2 + 0] = PREC ? rz : rr;
        a.partial[(int64_t)b * 2 + 1] = rr;
    }
}

// z = M^-1 r (cg_jacobi8) of the stored residual of every block of a live geometry, for
// the start of CG and after a residual replacement or rescaling; partial (r.z, r.r).
template <typename T>
__global__ __launch_bounds__(256) void k_cg_prec8(CgArgs a)
{
    __shared__ float tile[4][100];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int b = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + wv);
    if (b >= a.nb) return;
    const BlockInfo bi = a.info[b];
    int bx, by, bz, gid;
    block_pos(bi, &bx, &by, &bz, &gid);
    if (!geom_live<8>(a, gid)) {
        if (lane == 0) {
            a.partial[(int64_t)b * 2 + 0] = 0.0;
            a.partial[(int64_t)b * 2 + 1] = 0.0;
        }
        return;
    }
    const int64_t base = (int64_t)b * 512;
    const int lx = lane & 7, ly = lane >> 3;
    const uint64_t *rec = a.mask + (int64_t)b * 16;
    const GeomInfo g = a.geom[gid];
    const int gx = bx * 8 + lx, gy = by * 8 + ly;
    const bool bnd = bx == 0 || by == 0 || bz == 0 || bx * 8 + 8 >= g.nx || by * 8 + 8 >= g.ny ||
                     bz * 8 + 8 >= g.nz;
    float rk[8], vk[8];
    double rr = 0.0;
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        const bool act = lane_bit(rec[z]);
        const unsigned code = act ? (unsigned)a.code[base + z * 64 + lane] : 0u;
        const float r = act ? rd_ld((const T *)a.r, base + z * 64 + lane) : 0.0f;
        unsigned onf = 0u;
        if (bnd)
            onf = (gx == 0 ? 1u : 0u) | (gx == g.nx - 1 ? 2u : 0u) | (gy == 0 ? 4u : 0u) |
                  (gy == g.ny - 1 ? 8u : 0u) | (bz * 8 + z == 0 ? 16u : 0u) |
                  (bz * 8 + z == g.nz - 1 ? 32u : 0u);
        const bool fr = (code & 64u) != 0u && (onf & a.dir) == 0u;
        rk[z] = fr ? r : 0.0f;
        vk[z] = fr ? cg_inv_count(code) : 0.0f;
        rr += (double)rk[z] * (double)rk[z];
    }
    float *ts = tile[wv];
    tile_ring_zero(ts, lx, ly);
    float zk[8];
    cg_jacobi8(ts, lx, ly, rk, vk, a.prec, zk);
    double rz = 0.0;
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        const float zs = rd_round<T>(zk[z]);
        rz += (double)rk[z] * (double)zs;
        if (sector_active<T>(rec[z], lane)) rd_st_keep((T *)a.z, base + z * 64 + lane, zk[z]);
    }
    rz = wave_sum(rz);
    rr = wave_sum(rr);
    if (lane == 0) {
        a.partial[(int64_t)b * 2 + 0] = rz;
        a.partial[(int64_t)b * 2 + 1] = rr;
    }
}

// x += alpha p, r -= alpha Ap on free voxels of live geometries; partial (r.r, r.r)
template <typename T, int B>
__global__ __launch_bounds__(256) void k_cg_update(CgArgs a)
{
    using K = Blk<B>;
    using C = Cfg<B>;
    const int sub = threadIdx.x / C::TPB, lt = threadIdx.x % C::TPB;
    const int b = blockIdx.x * C::BPW + sub;
    bool valid = b < a.nb;
    int gid = 0;
    BlockInfo bi = {};
    if (valid) {
        bi = a.info[b];
        int bx, by, bz;
        block_pos(bi, &bx, &by, &bz, &gid);
        valid = geom_live<B>(a, gid);
    }
    double rr = 0.0;
    if (valid) {
        const float alpha = (float)a.scal[gid * CG_NSCAL + CG_ALPHA];
        const uint64_t *rec = a.mask + (int64_t)b * K::MW;
        const GeomInfo g = a.geom[gid];
        for (int k = 0; k < C::VPT; ++k) {
            const int slot = lt + k * C::TPB;
            if (!own_bit<B>(rec, slot)) continue;
            int bx, by, bz, gg;
            block_pos(bi, &bx, &by, &bz, &gg);
            const int gx = bx * B + slot % B, gy = by * B + (slot / B) % B, gz = bz * B + slot / (B * B);
            if (on_dirichlet(a.dir, gx, gy, gz, g.nx, g.ny, g.nz)) continue;
            const int64_t i = (int64_t)b * K::NS + slot;
            const float p = rd_ld((const T *)a.p, i);
            const float ap = rd_ld((const T *)a.ap, i);
            const float r = fmaf(-alpha, ap, rd_ld((const T *)a.r, i));
            if (a.x64 && a.x64_direct) {  // p holds sigma p
                a.x64[i] = fma(a.scal[gid * CG_NSCAL + CG_ALPHA] / a.scal[gid * CG_NSCAL + CG_SIGMA], (double)p,
                               a.x64[i]);
            } else {
                rd_st_keep((T *)a.x, i, fmaf(alpha, p, rd_ld((const T *)a.x, i)));
            }
            rd_st_keep((T *)a.r, i, r);
            const float rs = rd_ld((const T *)a.r, i);  // the stored (rounded) residual
            rr += (double)rs * (double)rs;
        }
    }
    block_sum2<B>(rr, rr, a.partial, b, b < a.nb);
}

// p = r + beta p on free voxels of live geometries
template <typename T, int B>
__global__ __launch_bounds__(256) void k_cg_pupdate(CgArgs a)
{
    using K = Blk<B>;
    using C = Cfg<B>;
    const int sub = threadIdx.x / C::TPB, lt = threadIdx.x % C::TPB;
    const int b = blockIdx.x * C::BPW + sub;
    if (b >= a.nb) return;
    const BlockInfo bi = a.info[b];
    int bx, by, bz, gid;
    block_pos(bi, &bx, &by, &bz, &gid);
    if (!geom_live<B>(a, gid)) return;
    const float beta = (float)a.scal[gid * CG_NSCAL + CG_BETA];
    const GeomInfo g = a.geom[gid];
    const uint64_t *rec = a.mask + (int64_t)b * K::MW;
    for (int k = 0; k < C::VPT; ++k) {
        const int slot = lt + k * C::TPB;
        if (!own_bit<B>(rec, slot)) continue;
        const int gx = bx * B + slot % B, gy = by * B + (slot / B) % B, gz = bz * B + slot / (B * B);
        if (on_dirichlet(a.dir, gx, gy, gz, g.nx, g.ny, g.nz)) continue;
        const int64_t i = (int64_t)b * K::NS + slot;
        rd_st_keep((T *)a.p, i, fmaf(beta, rd_ld((const T *)a.p, i), rd_ld((const T *)a.r, i)));
    }
}

// Per-geometry sums of the per-block partial pairs: geometry g owns blocks
// [block0_g, block0_{g+1}); one workgroup per geometry, fixed summation order.
// dst[g*CG_NSCAL + slot0 + k] = sum (k = 0, 1; slot < 0 skips that lane); then, for a
// live geometry, the scalar recurrence `mode`: 0 alpha = rr / pAp; 1 beta = rr_new / rr,
// rr = rr_new; 2 rr = rr_new (start); -1 none; -2 none, and only geometries whose CG_REPL
// slot is set are written.
__global__ __launch_bounds__(256) void k_cg_segsum(const double *part, const GeomInfo *geom,
                                                   int ngeom, int nb, double *scal, int slot0,
                                                   int slot1, int mode)
{
    __shared__ double sh[2][256];
    const int g = blockIdx.x;
    if (g >= ngeom) return;
    const int lo = geom[g].block0;
    const int hi = g + 1 < ngeom ? geom[g + 1].block0 : nb;
    double s0 = 0.0, s1 = 0.0;
    // thread t adds rows t, t + 256, ... in that order; eight rows' loads are issued
    // before their adds, so a long segment is not one load latency per row
    int i = lo + (int)threadIdx.x;
    for (; i + 7 * 256 < hi; i += 8 * 256) {
        double v0[8], v1[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            v0[k] = part[(int64_t)(i + k * 256) * 2 + 0];
            v1[k] = part[(int64_t)(i + k * 256) * 2 + 1];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            s0 += v0[k];
            s1 += v1[k];
        }
    }
    for (; i < hi; i += 256) {
        s0 += part[(int64_t)i * 2 + 0];
        s1 += part[(int64_t)i * 2 + 1];
    }
    sh[0][threadIdx.x] = s0;
    sh[1][threadIdx.x] = s1;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double *s = scal + g * CG_NSCAL;
        if (mode == -2 && s[CG_REPL] == 0.0) return;  // only the geometries just replaced
        if (slot0 >= 0) s[slot0] = sh[0][0];
        if (slot1 >= 0) s[slot1] = sh[1][0];
        // then the scalar recurrence of this geometry (live ones only)
        if (mode >= 0 && s[CG_DONE] == 0.0) {
            if (mode == 0) {
                s[CG_ALPHA] = s[CG_PAP] > 0.0 ? s[CG_RR] / s[CG_PAP] : 0.0;
            } else if (mode == 1) {
                s[CG_BETA] = s[CG_RR] > 0.0 ? s[CG_RRNEW] / s[CG_RR] : 0.0;
                s[CG_RR] = s[CG_RRNEW];
            } else {
                s[CG_RR] = s[CG_RRNEW];
            }
        }
    }
}


// ---- initial guess of the unit-drop problem: 6-connected clusters on the GPU ----
// Lock-free union-find over the slots, after the hooking and pointer-jumping scheme of
// ECL-CC (Jaiganesh and Burtscher, 2018): par[i] starts at i; every active voxel unites
// with its active +x, +y, +z neighbours by hooking the larger of the two roots under
// the smaller with a compare-and-swap.  Every parent index is therefore below its
// child's, each chain strictly decreases (every loop ends), and each cluster ends up
// rooted at its smallest slot index whatever the order of the unions.  All accesses to
// par while unions run are device-scope atomics, so workgroups on different XCDs agree
// on one order of updates per slot.
__device__ __forceinline__ uint32_t uf_load(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t uf_find(uint32_t *par, uint32_t x)
{
    uint32_t cur = uf_load(par + x);
    if (cur == x) return x;
    uint32_t prev = x, next;
    while (cur > (next = uf_load(par + cur))) {
        atomicMin(par + prev, next);  // path halving: a closer ancestor (a smaller index)
        prev = cur;
        cur = next;
    }
    return cur;
}

__device__ __forceinline__ void uf_unite(uint32_t *par, uint32_t a, uint32_t b)
{
    uint32_t ra = uf_find(par, a), rb = uf_find(par, b);
    while (ra != rb) {
        if (ra < rb) {
            const uint32_t t = ra;
            ra = rb;
            rb = t;
        }
        const uint32_t old = atomicCAS(par + ra, ra, rb);  // hook ra under rb if ra is a root
        if (old == ra) return;
        ra = old;  // ra was hooked meanwhile: go on from its parent (ra + rb decreases)
    }
}

__global__ __launch_bounds__(256) void k_lab_init(uint32_t *par, int64_t nslots)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < nslots) par[i] = (uint32_t)i;
}

// every active slot unites with its active +x, +y, +z neighbours (each pair once)
template <int B>
__global__ __launch_bounds__(256) void k_lab_unite(const BlockInfo *info, const uint8_t *code,
                                                   int64_t nslots, uint32_t *par)
{
    constexpr int NS = B * B * B;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= nslots) return;
    const unsigned cd = code[i];
    if (!(cd & 64u)) return;
    const int64_t b = i / NS;
    const int slot = (int)(i % NS);
    const int lc[3] = {slot % B, (slot / B) % B, slot / (B * B)};
    const int stride[3] = {1, B, B * B};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (!((cd >> (2 * d + 1)) & 1u)) continue;  // active neighbour in the box: its block exists
        const int64_t j = lc[d] < B - 1 ? i + stride[d]
                                        : (int64_t)info[b].nbr[2 * d + 1] * NS + slot - (B - 1) * stride[d];
        uf_unite(par, (uint32_t)i, (uint32_t)j);
    }
}

// B = 8 in two passes, so that most unions stay inside a workgroup: (1) every block
// labels its own active voxels in LDS by min-label propagation along its in-block
// edges (each label ends at the smallest slot of its in-block component) and writes
// par[i] = block base + that slot (a root's parent is itself; every parent index is at
// most its child's, as the global unions require); (2) only the pairs across the +x, +y
// and +z faces of each block are united globally (uf_unite), 192 candidate pairs per
// block instead of three per voxel.
__global__ __launch_bounds__(256) void k_lab_local8(const uint8_t *code, uint32_t *par)
{
    __shared__ uint16_t lab[512];
    __shared__ int changed;
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * 512;
    unsigned cd[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int s = t + 256 * k;
        cd[k] = code[base + s];
        lab[s] = (cd[k] & 64u) ? (uint16_t)s : (uint16_t)0xffff;
    }
    for (int it = 0; it < 512; ++it) {  // each pass lowers a label or ends the loop
        if (t == 0) changed = 0;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int s = t + 256 * k;
            if (!(cd[k] & 64u)) continue;
            const int l[3] = {s & 7, (s >> 3) & 7, s >> 6};
            unsigned m = lab[s];
#pragma unroll
            for (int d = 0; d < 6; ++d) {
                const int a = d >> 1;
                const bool up = d & 1;
                if (!((cd[k] >> d) & 1u) || (up ? l[a] == 7 : l[a] == 0)) continue;  // not in this block
                const int st = a == 0 ? 1 : a == 1 ? 8 : 64;
                const unsigned q = lab[up ? s + st : s - st];
                m = q < m ? q : m;
            }
            if (m < lab[s]) {
                lab[s] = (uint16_t)m;
                changed = 1;
            }
        }
        __syncthreads();
        const int c = changed;
        __syncthreads();
        if (!c) break;
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int s = t + 256 * k;
        par[base + s] = (uint32_t)(base + ((cd[k] & 64u) ? lab[s] : s));
    }
}

__global__ __launch_bounds__(256) void k_lab_faces8(const BlockInfo *info, const uint8_t *code, uint32_t *par)
{
    const int t = threadIdx.x;
    if (t >= 192) return;
    const int64_t b = blockIdx.x;
    const int a = t >> 6, u = t & 7, v = (t >> 3) & 7;  // face +x (a = 0), +y (1), +z (2)
    const int s = a == 0 ? (v * 8 + u) * 8 + 7 : a == 1 ? (v * 8 + 7) * 8 + u : (7 * 8 + v) * 8 + u;
    const int64_t i = b * 512 + s;
    const unsigned cd = code[i];
    if (!(cd & 64u) || !((cd >> (2 * a + 1)) & 1u)) return;  // active neighbour across the face
    const int st = a == 0 ? 1 : a == 1 ? 8 : 64;
    const int64_t j = (int64_t)info[b].nbr[2 * a + 1] * 512 + s - 7 * st;
    uf_unite(par, (uint32_t)i, (uint32_t)j);
}

// coordinate of slot i along `axis` and the extent of its geometry along it
template <int B>
__device__ __forceinline__ void lab_coord(const BlockInfo *info, const GeomInfo *geom, int64_t i, int axis,
                                          int *c, int *n, int *gid)
{
    constexpr int NS = B * B * B;
    const int slot = (int)(i % NS);
    int bx, by, bz;
    block_pos(info[i / NS], &bx, &by, &bz, gid);
    const GeomInfo g = geom[*gid];
    *c = axis == 0 ? bx * B + slot % B : axis == 1 ? by * B + (slot / B) % B : bz * B + slot / (B * B);
    *n = axis == 0 ? g.nx : axis == 1 ? g.ny : g.nz;
}

// par[i] = root of i (active slots); flags of the roots whose cluster touches the
// inlet plane (fin) or the outlet plane (fout)
template <int B>
__global__ __launch_bounds__(256) void k_lab_touch(const BlockInfo *info, const uint8_t *code,
                                                   const GeomInfo *geom, int64_t nslots, int axis,
                                                   uint32_t *par, uint8_t *fin, uint8_t *fout)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= nslots || !(code[i] & 64u)) return;
    const uint32_t r = uf_find(par, (uint32_t)i);
    __hip_atomic_store(par + i, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int c, n, gid;
    lab_coord<B>(info, geom, i, axis, &c, &n, &gid);
    if (c == 0) fin[r] = 1;  // every writer stores the same byte value
    if (c == n - 1) fout[r] = 1;
}

// x on every slot: the inlet plane 1, the outlet plane 0; inside, the linear ramp
// 1 - c/(n-1) on clusters touching both planes, 1 on clusters touching only the inlet
// (their exact solution), 0 on the others (exact too: a floating cluster's residual
// is zero, so CG never moves it); inactive slots 0.  perc[g] = 1 when a cluster of
// geometry g touches both planes.
template <typename T, int B>
__global__ __launch_bounds__(256) void k_lab_guess(const BlockInfo *info, const uint8_t *code,
                                                   const GeomInfo *geom, int64_t nslots, int axis,
                                                   const uint32_t *par, const uint8_t *fin,
                                                   const uint8_t *fout, T *x, double *X, uint32_t *perc)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= nslots) return;
    double v = 0.0;
    if (code[i] & 64u) {
        int c, n, gid;
        lab_coord<B>(info, geom, i, axis, &c, &n, &gid);
        const uint32_t r = par[i];
        const int t = (int)fin[r] | ((int)fout[r] << 1);
        if (c == 0) v = 1.0;
        else if (c == n - 1) v = 0.0;
        else if (t == 3) v = 1.0 - (double)c / (double)(n - 1);
        else v = t == 1 ? 1.0 : 0.0;
        if (t == 3) perc[gid] = 1u;
    }
    X[i] = v;  // the FP64 iterate starts at the exact ramp
    rd_st_keep(x, i, (float)v);
}

// ---- FP64 iterate of the steady state -------------------------------------
// CG keeps its iterate X in FP64 (the vectors r, p stay in the storage type): the true
// residual b - A X is evaluated in FP64 at every check and replaces the recursive one
// when they drift apart.  The generic kernels below take one thread per slot and read
// neighbours directly (they run a few times per solve).

// slot index of the neighbour of slot i across direction d (order -x,+x,-y,+y,-z,+z);
// the caller has checked that the neighbour is active (so its block exists)
template <int B>
__device__ __forceinline__ int64_t ir_nbr(const BlockInfo *info, int64_t i, int d)
{
    constexpr int NS = B * B * B;
    const int64_t b = i / NS;
    const int slot = (int)(i % NS);
    const int l = d < 2 ? slot % B : d < 4 ? (slot / B) % B : slot / (B * B);
    const int st = d < 2 ? 1 : d < 4 ? B : B * B;
    if (d & 1) return l < B - 1 ? i + st : (int64_t)info[b].nbr[d] * NS + slot - (B - 1) * st;
    return l > 0 ? i - st : (int64_t)info[b].nbr[d] * NS + slot + (B - 1) * st;
}

template <int B>
__device__ __forceinline__ void ir_pos(const BlockInfo *info, const GeomInfo *geom, int64_t i, int *gx, int *gy,
                                       int *gz, GeomInfo *g)
{
    constexpr int NS = B * B * B;
    const int slot = (int)(i % NS);
    int bx, by, bz, gid;
    block_pos(info[i / NS], &bx, &by, &bz, &gid);
    *g = geom[gid];
    *gx = bx * B + slot % B;
    *gy = by * B + (slot / B) % B;
    *gz = bz * B + slot / (B * B);
}

// r = b - A X on free voxels in FP64 from the FP64 iterate X, with the Dirichlet values
// held in X: r_p = sum over active neighbours q of (X_q - X_p) (difference form, order
// -x,+x,-y,+y,-z,+z); b_p = sum of the Dirichlet neighbours' X_q.  Per-block FP64
// partials (r.r, b.b) as the other CG kernels write them.  store 1: r rounded to the
// storage type becomes the CG residual and direction (r and p; 0 off the free voxels);
// store 2: sigma r replaces the residual (residual replacement) and p is rescaled from
// sigma_prev to sigma (powers of 2: exact), so that 16-bit vectors stay in range as the
// residual shrinks; store 3: r and p are only rescaled.  With store 2 or 3 each geometry
// takes its own choice from its CG_REPL slot (2, 3, or 0: untouched, partials 0), so a
// batch replaces only the residuals of the geometries that need it.  With store 2 or 3 the
// first partial is that of the stored r.
template <typename T, int B>
__global__ __launch_bounds__(256) void k_res64(CgArgs a, int store)
{
    using C = Cfg<B>;
    constexpr int NS = B * B * B;
    const int sub = threadIdx.x / C::TPB, lt = threadIdx.x % C::TPB;
    const int b = blockIdx.x * C::BPW + sub;
    double rr = 0.0, bb = 0.0;
    if (b < a.nb) {
        int bx, by, bz, gid;
        block_pos(a.info[b], &bx, &by, &bz, &gid);
        // store >= 2: each geometry's own choice (CG_REPL: 2 replace, 3 rescale, 0 none)
        const int st = store >= 2 ? (int)a.scal[gid * CG_NSCAL + CG_REPL] : store;
        const double sig = st >= 2 ? a.scal[gid * CG_NSCAL + CG_SIGMA] : 1.0;
        const float pscale = st >= 2 ? (float)(sig / a.scal[gid * CG_NSCAL + CG_SIGMA_PREV]) : 1.0f;
        const bool untouched = store >= 2 && st == 0;
        for (int k = 0; k < (untouched ? 0 : C::VPT); ++k) {
            const int64_t i = (int64_t)b * NS + lt + k * C::TPB;
            const unsigned cd = a.code[i];
            if (st == 3) {  // rescale only
                const float rs = rd_round<T>(pscale * rd_ld((const T *)a.r, i));
                rr += (double)rs * (double)rs;
                rd_st_keep((T *)a.r, i, rs);
                rd_st_keep((T *)a.p, i, pscale * rd_ld((const T *)a.p, i));
                continue;
            }
            float out = 0.0f;
            if (cd & 64u) {
                int gx, gy, gz;
                GeomInfo g;
                ir_pos<B>(a.info, a.geom, i, &gx, &gy, &gz, &g);
                if (!on_dirichlet(a.dir, gx, gy, gz, g.nx, g.ny, g.nz)) {
                    const double xp = a.x64[i];
                    double s = 0.0, bp = 0.0;
#pragma unroll
                    for (int d = 0; d < 6; ++d) {
                        if (!((cd >> d) & 1u)) continue;
                        const double xq = a.x64[ir_nbr<B>(a.info, i, d)];
                        s += xq - xp;
                        const int ex = d == 0 ? -1 : d == 1 ? 1 : 0, ey = d == 2 ? -1 : d == 3 ? 1 : 0,
                                  ez = d == 4 ? -1 : d == 5 ? 1 : 0;
                        if (on_dirichlet(a.dir, gx + ex, gy + ey, gz + ez, g.nx, g.ny, g.nz)) bp += xq;
                    }
                    out = (float)(sig * s);
                    if (st == 2) {
                        const double rs = (double)rd_round<T>(out);
                        rr += rs * rs;
                    } else {
                        rr += s * s;
                    }
                    bb += bp * bp;
                }
            }
            if (st == 1 || st == 2) rd_st_keep((T *)a.r, i, out);
            if (st == 1) rd_st_keep((T *)a.p, i, out);
            if (st == 2 && pscale != 1.0f) rd_st_keep((T *)a.p, i, pscale * rd_ld((const T *)a.p, i));
        }
    }
    block_sum2<B>(rr, bb, a.partial, b, b < a.nb);
}

// The FP64 true residual of the iterate X + x / sigma (x: the FP32 updates not yet
// folded, SPLIT) or X, for 8^3 blocks in the column form: one wave per block, lane
// (lx, ly) walking its z-column, X staged plane by plane in an FP64 LDS tile.  Same sums
// as k_res64 (difference form, order -x,+x,-y,+y,-z,+z); read-only; per-block partials
// (r.r, b.b).
template <typename T, bool SPLIT>
__global__ __launch_bounds__(256) void k_res64c(CgArgs a)
{
    __shared__ double tile[4][100];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int b = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + wv);
    if (b >= a.nb) return;
    const BlockInfo bi = a.info[b];
    int bx, by, bz, gid;
    block_pos(bi, &bx, &by, &bz, &gid);
    const double inv_s = SPLIT ? 1.0 / a.scal[gid * CG_NSCAL + CG_SIGMA] : 0.0;
    const T *xv = (const T *)a.x;
    const int64_t base = (int64_t)b * 512;
    const int lx = lane & 7, ly = lane >> 3;
    const uint64_t *rec = a.mask + (int64_t)b * 16;
    uint64_t Wo[8], Wf[6];
#pragma unroll
    for (int z = 0; z < 8; ++z) Wo[z] = rec[z];
#pragma unroll
    for (int f = 0; f < 6; ++f) Wf[f] = rec[8 + f];
    double c[8], hv[6];
    unsigned cd[8];
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        const int64_t i = base + z * 64 + lane;
        c[z] = 0.0;
        cd[z] = 0u;
        if (lane_bit(Wo[z])) {
            c[z] = a.x64[i];
            if (SPLIT) c[z] += (double)rd_ld(xv, i) * inv_s;
            cd[z] = (unsigned)a.code[i];
        }
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        int ns;
        switch (f) {
        case 0: ns = (ly * 8 + lx) * 8 + 7; break;
        case 1: ns = (ly * 8 + lx) * 8 + 0; break;
        case 2: ns = (ly * 8 + 7) * 8 + lx; break;
        case 3: ns = (ly * 8 + 0) * 8 + lx; break;
        case 4: ns = (7 * 8 + ly) * 8 + lx; break;
        default: ns = (0 * 8 + ly) * 8 + lx; break;
        }
        const int n = bi.nbr[f];
        const int64_t hb = (int64_t)(n >= 0 ? n : b) * 512 + ns;
        hv[f] = 0.0;
        if (lane_bit(Wf[f])) {
            hv[f] = a.x64[hb];
            if (SPLIT) hv[f] += (double)rd_ld(xv, hb) * inv_s;
        }
    }
    const GeomInfo g = a.geom[gid];
    const int gx = bx * 8 + lx, gy = by * 8 + ly;
    const bool bnd = bx == 0 || by == 0 || bz == 0 || bx * 8 + 8 >= g.nx || by * 8 + 8 >= g.ny ||
                     bz * 8 + 8 >= g.nz;
    double *ts = tile[wv];
    double rr = 0.0, bb = 0.0;
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        ts[(ly + 1) * 10 + (lx + 1)] = c[z];
        if (ly == z) {
            ts[(lx + 1) * 10 + 0] = hv[0];
            ts[(lx + 1) * 10 + 9] = hv[1];
            ts[0 * 10 + (lx + 1)] = hv[2];
            ts[9 * 10 + (lx + 1)] = hv[3];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const unsigned code = cd[z];
        const int gz = bz * 8 + z;
        const unsigned onf = bnd ? ((gx == 0 ? 1u : 0u) | (gx == g.nx - 1 ? 2u : 0u) | (gy == 0 ? 4u : 0u) |
                                    (gy == g.ny - 1 ? 8u : 0u) | (gz == 0 ? 16u : 0u) | (gz == g.nz - 1 ? 32u : 0u))
                                 : 0u;
        if ((code & 64u) && !(onf & a.dir)) {
            const double *q = &ts[(ly + 1) * 10 + (lx + 1)];
            const double nv[6] = {q[-1], q[1], q[-10], q[10], z == 0 ? hv[4] : c[z > 0 ? z - 1 : 0],
                                  z == 7 ? hv[5] : c[z < 7 ? z + 1 : 7]};
            double s = 0.0, bp = 0.0;
#pragma unroll
            for (int d = 0; d < 6; ++d) {
                if (!((code >> d) & 1u)) continue;
                s += nv[d] - c[z];
                if (bnd) {
                    const int ex = d == 0 ? -1 : d == 1 ? 1 : 0, ey = d == 2 ? -1 : d == 3 ? 1 : 0,
                              ez = d == 4 ? -1 : d == 5 ? 1 : 0;
                    if (on_dirichlet(a.dir, gx + ex, gy + ey, gz + ez, g.nx, g.ny, g.nz)) bp += nv[d];
                }
            }
            rr += s * s;
            bb += bp * bp;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    rr = wave_sum(rr);
    bb = wave_sum(bb);
    if (lane == 0) {
        a.partial[(int64_t)b * 2 + 0] = rr;
        a.partial[(int64_t)b * 2 + 1] = bb;
    }
}

// X += x / sigma of the slot's geometry, then x = 0 (every slot): the updates that x
// accumulated since the last check join the FP64 iterate
template <typename T, int B>
__global__ __launch_bounds__(256) void k_ir_fold(const BlockInfo *info, const double *scal, int64_t nslots,
                                                 double *X, T *x)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= nslots) return;
    const float v = rd_ld((const T *)x, i);
    if (v != 0.0f) {
        int bx, by, bz, gid;
        block_pos(info[i / (B * B * B)], &bx, &by, &bz, &gid);
        X[i] += (double)v / scal[gid * CG_NSCAL + CG_SIGMA];
        rd_st_keep(x, i, 0.0f);
    }
}

// x = X rounded to the storage type, every slot
template <typename T>
__global__ __launch_bounds__(256) void k_ir_store(int64_t nslots, const double *X, T *x)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < nslots) rd_st_keep(x, i, (float)X[i]);
}

// FP64 flux through the two Dirichlet planes of the FP64 iterate: per-block partials
// (sum over inlet Dirichlet voxels p and their free neighbours q of X_p - X_q, the same
// over the outlet), in the block layout of the other CG partials.
template <int B>
__global__ __launch_bounds__(256) void k_flux64(CgArgs a, int inlet_face)
{
    using C = Cfg<B>;
    constexpr int NS = B * B * B;
    const int sub = threadIdx.x / C::TPB, lt = threadIdx.x % C::TPB;
    const int b = blockIdx.x * C::BPW + sub;
    double qin = 0.0, qout = 0.0;
    if (b < a.nb) {
        for (int k = 0; k < C::VPT; ++k) {
            const int64_t i = (int64_t)b * NS + lt + k * C::TPB;
            const unsigned cd = a.code[i];
            if (!(cd & 64u)) continue;
            int gx, gy, gz;
            GeomInfo g;
            ir_pos<B>(a.info, a.geom, i, &gx, &gy, &gz, &g);
            const bool on_in = on_dirichlet(1u << inlet_face, gx, gy, gz, g.nx, g.ny, g.nz);
            const bool on_out = !on_in && on_dirichlet(1u << (inlet_face + 1), gx, gy, gz, g.nx, g.ny, g.nz);
            if (!on_in && !on_out) continue;
            const double xp = a.x64[i];
            double q = 0.0;
#pragma unroll
            for (int d = 0; d < 6; ++d) {
                if (!((cd >> d) & 1u)) continue;
                const int ex = d == 0 ? -1 : d == 1 ? 1 : 0, ey = d == 2 ? -1 : d == 3 ? 1 : 0,
                          ez = d == 4 ? -1 : d == 5 ? 1 : 0;
                if (on_dirichlet(a.dir, gx + ex, gy + ey, gz + ez, g.nx, g.ny, g.nz)) continue;
                q += xp - a.x64[ir_nbr<B>(a.info, i, d)];
            }
            if (on_in) qin += q;
            else qout += q;
        }
    }
    block_sum2<B>(qin, qout, a.partial, b, b < a.nb);
}

template <int B>
int groups(int nb) { return (nb + Cfg<B>::BPW - 1) / Cfg<B>::BPW; }

}  // namespace

#define CG_DISPATCH(storage, B, KERNEL, grid, stream, ...)                                         \
    do {                                                                                           \
        hipStream_t st_ = (hipStream_t)(stream);                                                   \
        if ((B) == 8) {                                                                            \
            if ((storage) == 0) hipLaunchKernelGGL((KERNEL<float, 8>), grid, dim3(256), 0, st_, __VA_ARGS__);      \
            else if ((storage) == 1) hipLaunchKernelGGL((KERNEL<bf16_t, 8>), grid, dim3(256), 0, st_, __VA_ARGS__); \
            else hipLaunchKernelGGL((KERNEL<_Float16, 8>), grid, dim3(256), 0, st_, __VA_ARGS__);                  \
        } else {                                                                                   \
            if ((storage) == 0) hipLaunchKernelGGL((KERNEL<float, 4>), grid, dim3(256), 0, st_, __VA_ARGS__);      \
            else if ((storage) == 1) hipLaunchKernelGGL((KERNEL<bf16_t, 4>), grid, dim3(256), 0, st_, __VA_ARGS__); \
            else hipLaunchKernelGGL((KERNEL<_Float16, 4>), grid, dim3(256), 0, st_, __VA_ARGS__);                  \
        }                                                                                          \
        return (int)hipGetLastError();                                                             \
    } while (0)

static dim3 grid_for(int B, int nb)
{
    return dim3((unsigned)std::max(1, B == 8 ? groups<8>(nb) : groups<4>(nb)));
}

int cg_launch_matvec(int storage, int B, const CgArgs &a, void *stream)
{
    CG_DISPATCH(storage, B, k_cg_matvec, grid_for(B, a.nb), stream, a);
}
int cg_launch_matvec_fused(int storage, const CgArgs &a, void *stream)
{
    const dim3 grid((unsigned)std::max(1, (a.nb + 3) / 4));
    hipStream_t st = (hipStream_t)stream;
    if (storage == 0) hipLaunchKernelGGL((k_cg_matvec8<float>), grid, dim3(256), 0, st, a);
    else if (storage == 1) hipLaunchKernelGGL((k_cg_matvec8<bf16_t>), grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_cg_matvec8<_Float16>), grid, dim3(256), 0, st, a);
    return (int)hipGetLastError();
}
int cg_launch_update(int storage, int B, const CgArgs &a, void *stream)
{
    if (B == 8) {  // column form with A p recomputed (the fused matvec does not store it)
        const dim3 grid((unsigned)std::max(1, (a.nb + 3) / 4));
        hipStream_t st = (hipStream_t)stream;
        const bool x64 = a.x64 && a.x64_direct, prec = a.prec > 0;
#define UPD8(T_)                                                                                   \
    do {                                                                                           \
        if (x64 && prec) hipLaunchKernelGGL((k_cg_update8<T_, true, true>), grid, dim3(256), 0, st, a);    \
        else if (x64) hipLaunchKernelGGL((k_cg_update8<T_, true, false>), grid, dim3(256), 0, st, a);      \
        else if (prec) hipLaunchKernelGGL((k_cg_update8<T_, false, true>), grid, dim3(256), 0, st, a);     \
        else hipLaunchKernelGGL((k_cg_update8<T_, false, false>), grid, dim3(256), 0, st, a);              \
    } while (0)
        if (storage == 0) UPD8(float);
        else if (storage == 1) UPD8(bf16_t);
        else UPD8(_Float16);
#undef UPD8
        return (int)hipGetLastError();
    }
    CG_DISPATCH(storage, B, k_cg_update, grid_for(B, a.nb), stream, a);
}
int cg_launch_prec(int storage, const CgArgs &a, void *stream)
{
    const dim3 grid((unsigned)std::max(1, (a.nb + 3) / 4));
    hipStream_t st = (hipStream_t)stream;
    if (storage == 0) hipLaunchKernelGGL((k_cg_prec8<float>), grid, dim3(256), 0, st, a);
    else if (storage == 1) hipLaunchKernelGGL((k_cg_prec8<bf16_t>), grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_cg_prec8<_Float16>), grid, dim3(256), 0, st, a);
    return (int)hipGetLastError();
}
int cg_launch_pupdate(int storage, int B, const CgArgs &a, void *stream)
{
    CG_DISPATCH(storage, B, k_cg_pupdate, grid_for(B, a.nb), stream, a);
}
int cg_launch_flux(int B, const CgArgs &a, int inlet_face, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    if (B == 8) hipLaunchKernelGGL(k_flux64<8>, grid_for(8, a.nb), dim3(256), 0, st, a, inlet_face);
    else hipLaunchKernelGGL(k_flux64<4>, grid_for(4, a.nb), dim3(256), 0, st, a, inlet_face);
    return (int)hipGetLastError();
}
int cg_launch_initial_guess(int storage, int B, const CgArgs &a, int axis, int64_t nslots, uint32_t *par,
                            uint8_t *flags, uint32_t *perc, void *stream)
{
    if (nslots <= 0) return 0;
    hipStream_t st = (hipStream_t)stream;
    const dim3 grid((unsigned)((nslots + 255) / 256));
    uint8_t *fin = flags, *fout = flags + nslots;
    if (B == 8) {
        const dim3 blocks((unsigned)(nslots / 512));
        hipLaunchKernelGGL(k_lab_local8, blocks, dim3(256), 0, st, a.code, par);
        hipLaunchKernelGGL(k_lab_faces8, blocks, dim3(256), 0, st, a.info, a.code, par);
        hipLaunchKernelGGL(k_lab_touch<8>, grid, dim3(256), 0, st, a.info, a.code, a.geom, nslots, axis, par, fin, fout);
        if (storage == 0)
            hipLaunchKernelGGL((k_lab_guess<float, 8>), grid, dim3(256), 0, st, a.info, a.code, a.geom, nslots, axis,
                               par, fin, fout, (float *)a.x, a.x64, perc);
        else if (storage == 1)
            hipLaunchKernelGGL((k_lab_guess<bf16_t, 8>), grid, dim3(256), 0, st, a.info, a.code, a.geom, nslots, axis,
                               par, fin, fout, (bf16_t *)a.x, a.x64, perc);
        else
            hipLaunchKernelGGL((k_lab_guess<_Float16, 8>), grid, dim3(256), 0, st, a.info, a.code, a.geom, nslots, axis,
                               par, fin, fout, (_Float16 *)a.x, a.x64, perc);
    } else {
        hipLaunchKernelGGL(k_lab_init, grid, dim3(256), 0, st, par, nslots);
        hipLaunchKernelGGL(k_lab_unite<4>, grid, dim3(256), 0, st, a.info, a.code, nslots, par);
        hipLaunchKernelGGL(k_lab_touch<4>, grid, dim3(256), 0, st, a.info, a.code, a.geom, nslots, axis, par, fin, fout);
        if (storage == 0)
            hipLaunchKernelGGL((k_lab_guess<float, 4>), grid, dim3(256), 0, st, a.info, a.code, a.geom, nslots, axis,
                               par, fin, fout, (float *)a.x, a.x64, perc);
        else if (storage == 1)
            hipLaunchKernelGGL((k_lab_guess<bf16_t, 4>), grid, dim3(256), 0, st, a.info, a.code, a.geom, nslots, axis,
                               par, fin, fout, (bf16_t *)a.x, a.x64, perc);
        else
            hipLaunchKernelGGL((k_lab_guess<_Float16, 4>), grid, dim3(256), 0, st, a.info, a.code, a.geom, nslots, axis,
                               par, fin, fout, (_Float16 *)a.x, a.x64, perc);
    }
    return (int)hipGetLastError();
}
int ir_rows(int64_t nslots) { return (int)((nslots + 255) / 256); }
int cg_launch_res64(int storage, int B, const CgArgs &a, int store, void *stream)
{
    if (B == 8 && store == 0) {  // the check: column form, read-only, of X + x / sigma when split
        const dim3 grid((unsigned)std::max(1, (a.nb + 3) / 4));
        hipStream_t st = (hipStream_t)stream;
        const bool split = !a.x64_direct;
#define RES64C(T_)                                                                                 \
    do {                                                                                           \
        if (split) hipLaunchKernelGGL((k_res64c<T_, true>), grid, dim3(256), 0, st, a);              \
        else hipLaunchKernelGGL((k_res64c<T_, false>), grid, dim3(256), 0, st, a);                  \
    } while (0)
        if (storage == 0) RES64C(float);
        else if (storage == 1) RES64C(bf16_t);
        else RES64C(_Float16);
#undef RES64C
        return (int)hipGetLastError();
    }
    CG_DISPATCH(storage, B, k_res64, grid_for(B, a.nb), stream, a, store);
}
int ir_launch_store(int storage, int64_t nslots, const double *X, void *x, void *stream)
{
    if (nslots <= 0) return 0;
    hipStream_t st = (hipStream_t)stream;
    const dim3 grid((unsigned)ir_rows(nslots));
    if (storage == 0) hipLaunchKernelGGL((k_ir_store<float>), grid, dim3(256), 0, st, nslots, X, (float *)x);
    else if (storage == 1) hipLaunchKernelGGL((k_ir_store<bf16_t>), grid, dim3(256), 0, st, nslots, X, (bf16_t *)x);
    else hipLaunchKernelGGL((k_ir_store<_Float16>), grid, dim3(256), 0, st, nslots, X, (_Float16 *)x);
    return (int)hipGetLastError();
}
int ir_launch_fold(int storage, int B, const CgArgs &a, int64_t nslots, void *stream)
{
    if (nslots <= 0) return 0;
    hipStream_t st = (hipStream_t)stream;
    const dim3 grid((unsigned)ir_rows(nslots));
#define IR_FOLD(T_, B_)                                                                             \
    hipLaunchKernelGGL((k_ir_fold<T_, B_>), grid, dim3(256), 0, st, a.info, (const double *)a.scal, nslots, a.x64, \
                       (T_ *)a.x)
    if (B == 8) {
        if (storage == 0) IR_FOLD(float, 8);
        else if (storage == 1) IR_FOLD(bf16_t, 8);
        else IR_FOLD(_Float16, 8);
    } else {
        if (storage == 0) IR_FOLD(float, 4);
        else if (storage == 1) IR_FOLD(bf16_t, 4);
        else IR_FOLD(_Float16, 4);
    }
#undef IR_FOLD
    return (int)hipGetLastError();
}
int cg_launch_segsum(const CgArgs &a, int slot0, int slot1, int mode, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    if (a.ngeom == 1 && a.mid && a.nb > 4096) {
        // one long block list: fixed row ranges over 256 workgroups, then their sums, then
        // the recurrence on that single row (one workgroup over millions of rows would
        // take as long as a matvec)
        double *sum = a.mid + 1024;
        const int e = rd_launch_finish_reduce(a.partial, a.nb, 2, a.mid, sum, stream);
        if (e) return e;
        hipLaunchKernelGGL(k_cg_segsum, dim3(1), dim3(256), 0, st, (const double *)sum, a.geom, 1, 1, a.scal, slot0,
                           slot1, mode);
        return (int)hipGetLastError();
    }
    hipLaunchKernelGGL(k_cg_segsum, dim3((unsigned)a.ngeom), dim3(256), 0, st, (const double *)a.partial, a.geom,
                       a.ngeom, a.nb, a.scal, slot0, slot1, mode);
    return (int)hipGetLastError();
}
