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
    if (threadIdx.x < 2) {
        const int l = threadIdx.x;
        a.partial[(int64_t)blockIdx.x * 2 + l] = ((wsum[0][l] + wsum[1][l]) + wsum[2][l]) + wsum[3][l];
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

// out[l] += sum over parts of part[part*nl + l] (fixed order), l < nl
__global__ __launch_bounds__(256) void k_sum_acc(const double *part, int nparts, int nl, double *out)
{
    __shared__ double sh[256];
    for (int l = 0; l < nl; ++l) {
        double s = 0.0;
        for (int i = threadIdx.x; i < nparts; i += 256) s += part[(int64_t)i * nl + l];
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[l] += sh[0];
        __syncthreads();
    }
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
    ADJ_DISPATCH(storage, B, k_adjoint, dim3((unsigned)adj_groups(B, a.nb)), stream, a);
}

int adj_launch_seed(int storage, int B, const AdjArgs &a, int mode, void *stream)
{
    ADJ_DISPATCH(storage, B, k_adj_seed, dim3((unsigned)a.nb), stream, a, mode);
}

int adj_launch_sum_acc(const double *part, int nparts, int nl, double *out, void *stream)
{
    hipLaunchKernelGGL(k_sum_acc, dim3(1), dim3(256), 0, (hipStream_t)stream, part, nparts, nl, out);
    return (int)hipGetLastError();
}
