// k_adjoint.hip -- discrete adjoint of the FTCS step for one species.
//
// The forward step on free voxels is c^{n+1} = J c^n + g with
//   J = I + alpha * L_f - (beta + gamma * n_wall) I,
// L_f the graph Laplacian among active voxels (the mirror rule makes it symmetric)
// and g the Dirichlet contribution.  J is symmetric, so the adjoint recursion
// lambda^n = J^T lambda^{n+1} is the forward step applied to lambda with every
// Dirichlet value set to 0 (lambda is 0 on Dirichlet and inactive voxels).  The
// same per-voxel update (rd_update) is used, so the adjoint step rounds like the
// forward one.  Fused with it are the FP64 gradient partials
//   dL/dD += <lambda^{n+1}, dt/dx^2 * sum_q (c^n_q - c^n_p)>
//   dL/dk += <lambda^{n+1}, -dt * c^n>           (k: first-order decay rate).
#include "rd_device.h"
#include "rd_adjoint.h"

namespace {

template <typename T, int B>
__global__ __launch_bounds__(256) void k_adjoint(AdjArgs a)
{
    using K = Blk<B>;
    using C = Cfg<B>;
    __shared__ float tl[C::BPW][1][K::TL];
    __shared__ float tc[C::BPW][1][K::TL];
    __shared__ uint64_t srec[C::BPW][K::MW];
    __shared__ double wsum[4][2];
    const int sub = threadIdx.x / C::TPB, lt = threadIdx.x % C::TPB;
    const int b = blockIdx.x * C::BPW + sub;
    const bool valid = b < a.nb;
    BlockInfo bi = {};
    if (valid) {
        bi = a.info[b];
        if (lt < K::MW) srec[sub][lt] = a.mask[(int64_t)b * K::MW + lt];
    }
    stage_tile<float, B>(tl[sub], a.lam_in, 0, 1, b, bi, lt, valid);
    stage_tile<T, B>(tc[sub], (const T *)a.c, 0, 1, b, bi, lt, valid);
    __syncthreads();
    double gD = 0.0, gk = 0.0;
    if (valid) {
        int bx, by, bz, gid;
        block_pos(bi, &bx, &by, &bz, &gid);
        const GeomInfo g = a.geom[gid];
        const uint64_t *rec = srec[sub];
        for (int k = 0; k < C::VPT; ++k) {
            const int slot = lt + k * C::TPB;
            const int lx = slot % B, ly = (slot / B) % B, lz = slot / (B * B);
            const int gx = bx * B + lx, gy = by * B + ly, gz = bz * B + lz;
            const int64_t i = (int64_t)b * K::NS + slot;
            const int t = K::tidx(lx, ly, lz);
            const bool act = own_bit<B>(rec, slot);
            float out = 0.0f;
            if (act) {
                int nwall = 0;
                const unsigned nbm = nb_bits<B>(rec, lx, ly, lz, gx, gy, gz, g.nx, g.ny, g.nz, &nwall);
                const float lp = tl[sub][0][t];
                if (on_dirichlet(a.coef.dir, gx, gy, gz, g.nx, g.ny, g.nz)) {
                    out = lp;  // stays 0
                } else {
                    const float *ts = tl[sub][0];
                    const float nbv[6] = {ts[t - 1], ts[t + 1], ts[t - K::E], ts[t + K::E],
                                          ts[t - K::E * K::E], ts[t + K::E * K::E]};
                    const float cen[1] = {lp};
                    out = rd_update<1>(lp, nbv, nbm, nwall, a.coef, cen);
                    // gradient partials with the forward state c^n
                    const float *tcs = tc[sub][0];
                    const float cc = tcs[t];
                    const float cnb[6] = {tcs[t - 1], tcs[t + 1], tcs[t - K::E], tcs[t + K::E],
                                          tcs[t - K::E * K::E], tcs[t + K::E * K::E]};
                    double lap = 0.0;
#pragma unroll
                    for (int d = 0; d < 6; ++d)
                        if ((nbm >> d) & 1u) lap += (double)cnb[d] - (double)cc;
                    gD += (double)lp * lap;
                    gk -= (double)lp * (double)cc;
                }
            }
            a.lam_out[i] = out;
        }
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double s0 = wave_sum(gD), s1 = wave_sum(gk);
    if (lane == 0) {
        wsum[wave][0] = s0;
        wsum[wave][1] = s1;
    }
    __syncthreads();
    if (threadIdx.x < 2) {  // this workgroup's accumulator, in step order
        const int l = threadIdx.x;
        a.partial[(int64_t)blockIdx.x * 2 + l] += ((wsum[0][l] + wsum[1][l]) + wsum[2][l]) + wsum[3][l];
    }
}

// The adjoint step for 8^3 blocks in the column form of the forward step: one wave per
// block (four per workgroup), lane (lx, ly) walking its z-column; lambda^{n+1} and c^n
// of the block and of its face halos are loaded under the activity predicates, the
// +-x / +-y neighbours of both go through one-plane LDS tiles.  lambda^n on free
// voxels is rd_update on lambda (the forward step with zero Dirichlet data), 0
// elsewhere; the gradient terms of the block are added, in step order, to its own
// FP64 accumulators partial[b][0..1] (one wave owns a block, so there is no race):
//   dL/dD: lambda^{n+1}_p * (sum of the six c^n neighbours - n_active * c^n_p)
//   dL/dk: -lambda^{n+1}_p * c^n_p                      (scaled on the host)
template <typename T>
__global__ __launch_bounds__(256) void k_adjoint8(AdjArgs a)
{
    __shared__ float tl[4][100], tc[4][100];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int b = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + wv);
    if (b >= a.nb) return;
    const BlockInfo bi = a.info[b];
    const T *cv = (const T *)a.c;
    const int64_t base = (int64_t)b * 512;
    const int lx = lane & 7, ly = lane >> 3;
    const uint64_t *rec = a.mask + (int64_t)b * 16;
    uint64_t Wo[8], Wf[6];
#pragma unroll
    for (int z = 0; z < 8; ++z) Wo[z] = rec[z];
#pragma unroll
    for (int f = 0; f < 6; ++f) Wf[f] = rec[8 + f];
    typedef typename RawOf<T>::type R;
    float lc[8], lh[6];
    R cc[8], ch[6];
    unsigned cd[8];
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        const bool act = (Wo[z] >> lane) & 1ull;
        lc[z] = ld_raw(a.lam_in, base + z * 64 + lane, act);
        cc[z] = ld_raw(cv, base + z * 64 + lane, act);
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
        const int64_t hb = (int64_t)(n >= 0 ? n : b) * 512 + ns;
        lh[f] = ld_raw(a.lam_in, hb, e);
        ch[f] = ld_raw(cv, hb, e);
    }
    float c[8], cs[6];
#pragma unroll
    for (int z = 0; z < 8; ++z) c[z] = from_raw<T>(cc[z]);
#pragma unroll
    for (int f = 0; f < 6; ++f) cs[f] = from_raw<T>(ch[f]);

    int bx, by, bz, gid;
    block_pos(bi, &bx, &by, &bz, &gid);
    const GeomInfo g = a.geom[gid];
    const int gx = bx * 8 + lx, gy = by * 8 + ly;
    const bool bnd = bx == 0 || by == 0 || bz == 0 || bx * 8 + 8 >= g.nx || by * 8 + 8 >= g.ny ||
                     bz * 8 + 8 >= g.nz;
    float *TL = tl[wv], *TC = tc[wv];
    double gD = 0.0, gk = 0.0;
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        TL[(ly + 1) * 10 + (lx + 1)] = lc[z];
        TC[(ly + 1) * 10 + (lx + 1)] = c[z];
        if (ly == z) {  // side halos of plane z (face coordinate v = z)
            TL[(lx + 1) * 10 + 0] = lh[0];
            TL[(lx + 1) * 10 + 9] = lh[1];
            TL[0 * 10 + (lx + 1)] = lh[2];
            TL[9 * 10 + (lx + 1)] = lh[3];
            TC[(lx + 1) * 10 + 0] = cs[0];
            TC[(lx + 1) * 10 + 9] = cs[1];
            TC[0 * 10 + (lx + 1)] = cs[2];
            TC[9 * 10 + (lx + 1)] = cs[3];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const unsigned code = cd[z], m = code & 63u;
        unsigned onf = 0u;
        if (bnd)
            onf = (gx == 0 ? 1u : 0u) | (gx == g.nx - 1 ? 2u : 0u) | (gy == 0 ? 4u : 0u) |
                  (gy == g.ny - 1 ? 8u : 0u) | (bz * 8 + z == 0 ? 16u : 0u) |
                  (bz * 8 + z == g.nz - 1 ? 32u : 0u);
        const bool fr = (code & 64u) != 0u && (onf & a.coef.dir) == 0u;
        const int nwall = __popc(~onf & ~m & 0x3fu);
        const int o = (ly + 1) * 10 + (lx + 1);
        const float lp = lc[z];
        const float nbl[6] = {TL[o - 1], TL[o + 1], TL[o - 10], TL[o + 10], z == 0 ? lh[4] : lc[z > 0 ? z - 1 : 0],
                              z == 7 ? lh[5] : lc[z < 7 ? z + 1 : 7]};
        const float cen[1] = {lp};
        const float lout = fr ? rd_update<1>(lp, nbl, m, nwall, a.coef, cen) : 0.0f;
        if (fr) {
            const double sc = (((((double)TC[o - 1] + (double)TC[o + 1]) + (double)TC[o - 10]) +
                                (double)TC[o + 10]) + (double)(z == 0 ? cs[4] : c[z > 0 ? z - 1 : 0])) +
                              (double)(z == 7 ? cs[5] : c[z < 7 ? z + 1 : 7]);
            const double lapc = sc - (double)__popc(m) * (double)c[z];
            gD += (double)lp * lapc;
            gk -= (double)lp * (double)c[z];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // lambda is FP32 and read under activity predicates: whole 128-byte sectors
        if (sector_active<float>(Wo[z], lane)) a.lam_out[base + z * 64 + lane] = lout;
    }
    gD = wave_sum(gD);
    gk = wave_sum(gk);
    if (lane == 0) {
        a.partial[(int64_t)b * 2 + 0] += gD;
        a.partial[(int64_t)b * 2 + 1] += gk;
    }
}

// lambda^N on free voxels: c^N - c* (mode 0, loss partial 1/2 (c^N - c*)^2) or the
// given dL/dc^N (mode 1); 0 on Dirichlet and inactive slots.
template <typename T, int B>
__global__ __launch_bounds__(256) void k_adj_seed(AdjArgs a, int mode)
{
    using K = Blk<B>;
    __shared__ double wsum[4];
    const int b = blockIdx.x;
    double loss = 0.0;
    if (b < a.nb) {
        const BlockInfo bi = a.info[b];
        int bx, by, bz, gid;
        block_pos(bi, &bx, &by, &bz, &gid);
        const GeomInfo g = a.geom[gid];
        const uint64_t *rec = a.mask + (int64_t)b * K::MW;
        for (int slot = threadIdx.x; slot < K::NS; slot += 256) {
            const int gx = bx * B + slot % B, gy = by * B + (slot / B) % B, gz = bz * B + slot / (B * B);
            const int64_t i = (int64_t)b * K::NS + slot;
            float l = 0.0f;
            if (own_bit<B>(rec, slot) && !on_dirichlet(a.coef.dir, gx, gy, gz, g.nx, g.ny, g.nz)) {
                if (mode == 0) {
                    const float d = rd_ld((const T *)a.c, i) - a.seed[i];
                    l = d;
                    loss += 0.5 * (double)d * (double)d;
                } else {
                    l = a.seed[i];
                }
            }
            a.lam_out[i] = l;
        }
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double s = wave_sum(loss);
    if (lane == 0) wsum[wave] = s;
    __syncthreads();
    if (threadIdx.x == 0) a.partial[b] = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
}


// Adjoint step with a diffusivity factor, one thread per slot (see AdjEArgs).  The
// lambda update mirrors the inhomogeneous forward step in FP32; the gradient terms are
// FP64.  Rows as in k_adjoint: one per workgroup (B = 8: one block, B = 4: four).
template <typename T, int B>
__global__ __launch_bounds__(256) void k_adjoint_e(AdjEArgs x)
{
    using C = Cfg<B>;
    constexpr int NS = B * B * B;
    const AdjArgs &a = x.a;
    __shared__ double wsum[4][2];
    const int sub = threadIdx.x / C::TPB, lt = threadIdx.x % C::TPB;
    const int b = blockIdx.x * C::BPW + sub;
    double gD = 0.0, gk = 0.0;
    if (b < a.nb) {
        const BlockInfo bi = a.info[b];
        int bx, by, bz, gid;
        block_pos(bi, &bx, &by, &bz, &gid);
        const GeomInfo g = a.geom[gid];
        const T *c = (const T *)a.c;
        for (int k = 0; k < C::VPT; ++k) {
            const int slot = lt + k * C::TPB;
            const int64_t i = (int64_t)b * NS + slot;
            const unsigned code = a.code[i];
            float out = 0.0f;
            if (code & 64u) {
                const int lx = slot % B, ly = (slot / B) % B, lz = slot / (B * B);
                const int gx = bx * B + lx, gy = by * B + ly, gz = bz * B + lz;
                const unsigned onf = (gx == 0 ? 1u : 0u) | (gx == g.nx - 1 ? 2u : 0u) | (gy == 0 ? 4u : 0u) |
                                     (gy == g.ny - 1 ? 8u : 0u) | (gz == 0 ? 16u : 0u) |
                                     (gz == g.nz - 1 ? 32u : 0u);
                const unsigned m = code & 63u;
                const int nwall = __popc(~onf & ~m & 0x3fu);
                const float lp = a.lam_in[i], ep = x.e[i];
                const double cp = (double)rd_ld(c, i);
                float laml = 0.0f;
                double lapc = 0.0, gsum = 0.0;
                const int stride[3] = {1, B, B * B};
                for (int d = 0; d < 6; ++d) {
                    if (!((m >> d) & 1u)) continue;
                    const int ax = d >> 1, l = ax == 0 ? lx : ax == 1 ? ly : lz;
                    const bool up = d & 1;
                    int64_t q;
                    if (up ? l < B - 1 : l > 0) q = i + (up ? stride[ax] : -stride[ax]);
                    else q = (int64_t)bi.nbr[d] * NS + slot + (up ? -(B - 1) : (B - 1)) * stride[ax];
                    const float lq = a.lam_in[q], eq = x.e[q];
                    const double cq = (double)rd_ld(c, q);
                    laml = fmaf(0.5f * (ep + eq), lq - lp, laml);
                    lapc += 0.5 * ((double)ep + (double)eq) * (cq - cp);
                    gsum += (cq - cp) * ((double)lp - (double)lq);
                }
                x.ge[i] += 0.5 * x.alpha * gsum;  // lambda is 0 on Dirichlet voxels
                if (!(onf & a.coef.dir)) {
                    gD += (double)lp * lapc;
                    gk -= (double)lp * cp;
                    const float r = fmaf(a.coef.alpha, laml, lp);
                    out = fmaf(-fmaf(a.coef.gamma, (float)nwall, a.coef.beta), lp, r);
                }
            }
            a.lam_out[i] = out;
        }
    }
    const int wave = threadIdx.x >> 6;
    const double s0 = wave_sum(gD), s1 = wave_sum(gk);
    if ((threadIdx.x & 63) == 0) {
        wsum[wave][0] = s0;
        wsum[wave][1] = s1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a.partial[(int64_t)blockIdx.x * 2 + 0] += ((wsum[0][0] + wsum[1][0]) + wsum[2][0]) + wsum[3][0];
        a.partial[(int64_t)blockIdx.x * 2 + 1] += ((wsum[0][1] + wsum[1][1]) + wsum[2][1]) + wsum[3][1];
    }
}

// Column form of k_adjoint_e for 8^3 blocks: one wave per block, lane (lx, ly) walking
// z, lambda / c / e planes staged in LDS with their side halos, the z neighbours in
// registers.  Per voxel the same operations in the same order as k_adjoint_e (dL/de and
// lambda are bitwise equal; the dL/dD and dL/dk rows are summed in another order).
// One row per block.
template <typename T>
__global__ __launch_bounds__(256) void k_adjoint8e(AdjEArgs x)
{
    __shared__ float tl[4][100], tc[4][100], te[4][100];
    const AdjArgs &a = x.a;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int b = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + wv);
    if (b >= a.nb) return;
    const BlockInfo bi = a.info[b];
    const T *cv = (const T *)a.c;
    const int64_t base = (int64_t)b * 512;
    const int lx = lane & 7, ly = lane >> 3;
    const uint64_t *rec = a.mask + (int64_t)b * 16;
    uint64_t Wo[8], Wf[6];
#pragma unroll
    for (int z = 0; z < 8; ++z) Wo[z] = rec[z];
#pragma unroll
    for (int f = 0; f < 6; ++f) Wf[f] = rec[8 + f];
    float lc[8], lh[6], ec[8], eh[6];
    float cc[8], ch[6];
    unsigned cd[8];
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        const bool act = (Wo[z] >> lane) & 1ull;
        const int64_t i = base + z * 64 + lane;
        lc[z] = act ? a.lam_in[i] : 0.0f;
        cc[z] = act ? rd_ld(cv, i) : 0.0f;
        ec[z] = act ? x.e[i] : 0.0f;
        cd[z] = act ? (unsigned)a.code[i] : 0u;
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
        const bool on = (Wf[f] >> lane) & 1ull;
        const int64_t h = (int64_t)(n >= 0 ? n : b) * 512 + ns;
        lh[f] = on ? a.lam_in[h] : 0.0f;
        ch[f] = on ? rd_ld(cv, h) : 0.0f;
        eh[f] = on ? x.e[h] : 0.0f;
    }
    int bx, by, bz, gid;
    block_pos(bi, &bx, &by, &bz, &gid);
    const GeomInfo g = a.geom[gid];
    const int gx = bx * 8 + lx, gy = by * 8 + ly;
    auto pix = [](int px, int py) { return (py + 1) * 10 + (px + 1); };
    double gD = 0.0, gk = 0.0;
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        tl[wv][pix(lx, ly)] = lc[z];
        tc[wv][pix(lx, ly)] = cc[z];
        te[wv][pix(lx, ly)] = ec[z];
        if (ly == z) {
            tl[wv][pix(-1, lx)] = lh[0]; tl[wv][pix(8, lx)] = lh[1];
            tl[wv][pix(lx, -1)] = lh[2]; tl[wv][pix(lx, 8)] = lh[3];
            tc[wv][pix(-1, lx)] = ch[0]; tc[wv][pix(8, lx)] = ch[1];
            tc[wv][pix(lx, -1)] = ch[2]; tc[wv][pix(lx, 8)] = ch[3];
            te[wv][pix(-1, lx)] = eh[0]; te[wv][pix(8, lx)] = eh[1];
            te[wv][pix(lx, -1)] = eh[2]; te[wv][pix(lx, 8)] = eh[3];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const unsigned code = cd[z];
        float out = 0.0f;
        if (code & 64u) {
            const int gz = bz * 8 + z;
            const unsigned onf = (gx == 0 ? 1u : 0u) | (gx == g.nx - 1 ? 2u : 0u) | (gy == 0 ? 4u : 0u) |
                                 (gy == g.ny - 1 ? 8u : 0u) | (gz == 0 ? 16u : 0u) | (gz == g.nz - 1 ? 32u : 0u);
            const unsigned m = code & 63u;
            const int nwall = __popc(~onf & ~m & 0x3fu);
            const int t = pix(lx, ly);
            const float lp = lc[z], ep = ec[z];
            const double cp = (double)cc[z];
            const float lnv[6] = {tl[wv][t - 1], tl[wv][t + 1], tl[wv][t - 10], tl[wv][t + 10],
                                  z == 0 ? lh[4] : lc[z > 0 ? z - 1 : 0], z == 7 ? lh[5] : lc[z < 7 ? z + 1 : 7]};
            const float cnv[6] = {tc[wv][t - 1], tc[wv][t + 1], tc[wv][t - 10], tc[wv][t + 10],
                                  z == 0 ? ch[4] : cc[z > 0 ? z - 1 : 0], z == 7 ? ch[5] : cc[z < 7 ? z + 1 : 7]};
            const float env[6] = {te[wv][t - 1], te[wv][t + 1], te[wv][t - 10], te[wv][t + 10],
                                  z == 0 ? eh[4] : ec[z > 0 ? z - 1 : 0], z == 7 ? eh[5] : ec[z < 7 ? z + 1 : 7]};
            float laml = 0.0f;
            double lapc = 0.0, gsum = 0.0;
#pragma unroll
            for (int d = 0; d < 6; ++d) {
                if (!((m >> d) & 1u)) continue;
                const float lq = lnv[d], eq = env[d];
                const double cq = (double)cnv[d];
                laml = fmaf(0.5f * (ep + eq), lq - lp, laml);
                lapc += 0.5 * ((double)ep + (double)eq) * (cq - cp);
                gsum += (cq - cp) * ((double)lp - (double)lq);
            }
            const int64_t i = base + z * 64 + lane;
            x.ge[i] += 0.5 * x.alpha * gsum;
            if (!(onf & a.coef.dir)) {
                gD += (double)lp * lapc;
                gk -= (double)lp * cp;
                const float r = fmaf(a.coef.alpha, laml, lp);
                out = fmaf(-fmaf(a.coef.gamma, (float)nwall, a.coef.beta), lp, r);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        a.lam_out[base + z * 64 + lane] = out;
    }
    gD = wave_sum(gD);
    gk = wave_sum(gk);
    if (lane == 0) {
        a.partial[(int64_t)b * 2 + 0] += gD;
        a.partial[(int64_t)b * 2 + 1] += gk;
    }
}

template <int B>
__global__ __launch_bounds__(256) void k_dense_f64(const BlockInfo *info, const uint8_t *code, const GeomInfo *geom,
                                                   int nb, const double *v, double *dense)
{
    constexpr int NS = B * B * B;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)nb * NS || !(code[i] & 64u)) return;
    const int b = (int)(i / NS), slot = (int)(i % NS);
    int bx, by, bz, gid;
    block_pos(info[b], &bx, &by, &bz, &gid);
    const GeomInfo g = geom[gid];
    dense[voxel_id(g, bx * B + slot % B, by * B + (slot / B) % B, bz * B + slot / (B * B))] = v[i];
}

}  // namespace

#define ADJ_DISPATCH(storage, B, KERNEL, grid, stream, ...)                                        \
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

int adj_groups(int B, int nb) { return B == 8 ? nb : (nb + 3) / 4; }

int adj_launch_step(int storage, int B, const AdjArgs &a, void *stream)
{
    if (B == 8) {  // column form, four blocks per workgroup, per-block accumulators
        const dim3 grid((unsigned)((a.nb + 3) / 4));
        hipStream_t st = (hipStream_t)stream;
        if (storage == 0) hipLaunchKernelGGL((k_adjoint8<float>), grid, dim3(256), 0, st, a);
        else if (storage == 1) hipLaunchKernelGGL((k_adjoint8<bf16_t>), grid, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_adjoint8<_Float16>), grid, dim3(256), 0, st, a);
        return (int)hipGetLastError();
    }
    ADJ_DISPATCH(storage, B, k_adjoint, dim3((unsigned)adj_groups(B, a.nb)), stream, a);
}

int adj_launch_seed(int storage, int B, const AdjArgs &a, int mode, void *stream)
{
    ADJ_DISPATCH(storage, B, k_adj_seed, dim3((unsigned)a.nb), stream, a, mode);
}

int adj_launch_step_e(int storage, int B, const AdjEArgs &x, int column, void *stream)
{
    if (x.a.nb <= 0) return 0;
    hipStream_t st = (hipStream_t)stream;
    const dim3 grid((unsigned)adj_groups(B, x.a.nb));
    if (B == 8 && column) {  // four blocks per workgroup, one row per block
        const dim3 g8((unsigned)((x.a.nb + 3) / 4));
        if (storage == 0) hipLaunchKernelGGL((k_adjoint8e<float>), g8, dim3(256), 0, st, x);
        else if (storage == 1) hipLaunchKernelGGL((k_adjoint8e<bf16_t>), g8, dim3(256), 0, st, x);
        else hipLaunchKernelGGL((k_adjoint8e<_Float16>), g8, dim3(256), 0, st, x);
    } else if (B == 8) {
        if (storage == 0) hipLaunchKernelGGL((k_adjoint_e<float, 8>), grid, dim3(256), 0, st, x);
        else if (storage == 1) hipLaunchKernelGGL((k_adjoint_e<bf16_t, 8>), grid, dim3(256), 0, st, x);
        else hipLaunchKernelGGL((k_adjoint_e<_Float16, 8>), grid, dim3(256), 0, st, x);
    } else {
        if (storage == 0) hipLaunchKernelGGL((k_adjoint_e<float, 4>), grid, dim3(256), 0, st, x);
        else if (storage == 1) hipLaunchKernelGGL((k_adjoint_e<bf16_t, 4>), grid, dim3(256), 0, st, x);
        else hipLaunchKernelGGL((k_adjoint_e<_Float16, 4>), grid, dim3(256), 0, st, x);
    }
    return (int)hipGetLastError();
}

int adj_launch_dense_f64(int B, const BlockInfo *info, const uint8_t *code, const GeomInfo *geom, int nb,
                         const double *v, double *dense, int64_t ndense, void *stream)
{
    int rc = rd_launch_fill_u32(dense, 0u, 2 * ndense, stream);
    if (rc != 0 || nb <= 0) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = (int64_t)nb * B * B * B;
    const dim3 grid((unsigned)((n + 255) / 256));
    if (B == 8) hipLaunchKernelGGL((k_dense_f64<8>), grid, dim3(256), 0, st, info, code, geom, nb, v, dense);
    else hipLaunchKernelGGL((k_dense_f64<4>), grid, dim3(256), 0, st, info, code, geom, nb, v, dense);
    return (int)hipGetLastError();
}
