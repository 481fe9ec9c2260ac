// k_step.hip -- the sparse-block FTCS step, its FP64 reductions and the dense <->
// block-major layout kernels, for gfx950 (wave64, 160 KB LDS per CU).
//
// Step kernel (paper: FTCS with the mirror rule applied inside the stencil,
// sections "Discretization and numerical methods" and "Parallel implementation"):
//   * B = 8: one 256-thread workgroup per block, two voxels per thread;
//     B = 4: one wave per block, four blocks per workgroup, one voxel per thread.
//   * The block and its six face halos (read through the neighbour list) are staged
//     as FP32 in an LDS tile of (B+2)^3 words per species; corners are unused.
//   * Activity of the six neighbours comes from the block's mask record (own bits
//     plus the neighbours' face bits), so no neighbour mask is read.
//   * Inactive slots are written as 0; Dirichlet voxels are copied through.
// The stencil is HBM-bound (about 2 FLOP per byte), so there is no MFMA here.
#include "rd_device.h"

namespace {

template <int B>
struct Cfg {
    static constexpr int BPW = B == 8 ? 1 : 4;  // blocks per workgroup
    static constexpr int TPB = 256 / BPW;       // threads per block
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

template <typename T, int B>
__global__ __launch_bounds__(256) void k_step(StepArgs a)
{
    using K = Blk<B>;
    using C = Cfg<B>;
    __shared__ float tile[C::BPW][RD_MAX_SPECIES][K::TL];

    const int sub = threadIdx.x / C::TPB;
    const int lt = threadIdx.x % C::TPB;
    const int grp = map_group(blockIdx.x, a.xcd_chunk);
    const int b = grp * C::BPW + sub;
    const bool valid = b < a.nb;
    const T *cin = (const T *)a.cin;
    T *cout = (T *)a.cout;

    BlockInfo bi = {};
    uint64_t rec[K::MW];
    if (valid) {
        bi = a.info[b];
#pragma unroll
        for (int w = 0; w < K::MW; ++w) rec[w] = a.mask[(int64_t)b * K::MW + w];
    } else {
#pragma unroll
        for (int w = 0; w < K::MW; ++w) rec[w] = 0;
    }
    stage_tile<T, B>(tile[sub], cin, a.sstride, a.S, b, bi, lt, valid);
    __syncthreads();
    if (!valid) return;

    int bx, by, bz, gid;
    block_pos(bi, &bx, &by, &bz, &gid);
    const GeomInfo g = a.geom[gid];
    const int64_t base = (int64_t)b * K::NS;
#pragma unroll
    for (int k = 0; k < C::VPT; ++k) {
        const int slot = lt + k * C::TPB;
        const int lx = slot % B, ly = (slot / B) % B, lz = slot / (B * B);
        const int gx = bx * B + lx, gy = by * B + ly, gz = bz * B + lz;
        const bool act = own_bit<B>(rec, slot);
        int nwall = 0;
        const unsigned nbm = act ? nb_bits<B>(rec, lx, ly, lz, gx, gy, gz, g.nx, g.ny, g.nz, &nwall)
                                 : 0u;
        const int t = K::tidx(lx, ly, lz);
        float cen[RD_MAX_SPECIES];
        for (int s = 0; s < a.S; ++s) cen[s] = tile[sub][s][t];
        for (int s = 0; s < a.S; ++s) {
            float r;
            if (!act) {
                r = 0.0f;
            } else if (on_dirichlet(a.coef[s].dir, gx, gy, gz, g.nx, g.ny, g.nz)) {
                r = cen[s];
            } else {
                const float *ts = tile[sub][s];
                const float nbv[6] = {ts[t - 1], ts[t + 1], ts[t - K::E], ts[t + K::E],
                                      ts[t - K::E * K::E], ts[t + K::E * K::E]};
                r = rd_update(cen[s], nbv, nbm, nwall, a.coef[s], cen, a.S);
            }
            if (a.sround) {
                const uint32_t step = *a.ctr + a.ctr_off;
                rd_st_sr(cout, s * a.sstride + base + slot, r,
                         sr_bits(base + slot, s, step, a.seed));
            } else {
                rd_st(cout, s * a.sstride + base + slot, r);
            }
        }
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
    const int b = blockIdx.x * C::BPW + sub;
    const bool valid = b < a.nb;
    const T *c = (const T *)a.c;

    BlockInfo bi = {};
    uint64_t rec[K::MW];
    if (valid) {
        bi = a.info[b];
#pragma unroll
        for (int w = 0; w < K::MW; ++w) rec[w] = a.mask[(int64_t)b * K::MW + w];
    } else {
#pragma unroll
        for (int w = 0; w < K::MW; ++w) rec[w] = 0;
    }
    const T *cs = c + a.s * a.sstride;
    stage_tile<T, B>(tile[sub], cs, 0, 1, b, bi, lt, valid);
    __syncthreads();

    double acc[RD_NRED];
#pragma unroll
    for (int l = 0; l < RD_NRED; ++l) acc[l] = 0.0;
    if (valid) {
        int bx, by, bz, gid;
        block_pos(bi, &bx, &by, &bz, &gid);
        const GeomInfo g = a.geom[gid];
        const double dx = a.dx, dx2 = dx * dx, dx3 = dx2 * dx;
#pragma unroll
        for (int k = 0; k < C::VPT; ++k) {
            const int slot = lt + k * C::TPB;
            const int lx = slot % B, ly = (slot / B) % B, lz = slot / (B * B);
            const int gx = bx * B + lx, gy = by * B + ly, gz = bz * B + lz;
            if (!own_bit<B>(rec, slot)) continue;
            int nwall = 0;
            const unsigned nbm = nb_bits<B>(rec, lx, ly, lz, gx, gy, gz, g.nx, g.ny, g.nz, &nwall);
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
                for (int d = 0; d < 6; ++d) {
                    if (!((nbm >> d) & 1u)) continue;
                    if (on_dirichlet(a.dir, gx + ddx[d], gy + ddy[d], gz + ddz[d], g.nx, g.ny, g.nz))
                        continue;
                    acc[1 + fq] += a.D * (u - (double)ts[t + off[d]]) * dx;
                }
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
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
    for (int l = 0; l < RD_NRED; ++l) {
        const double v = wave_sum(acc[l]);
        if (lane == 0) wsum[wave][l] = v;
    }
    __syncthreads();
    if (threadIdx.x < RD_NRED) {
        const int l = threadIdx.x;
        a.partial[(int64_t)blockIdx.x * RD_NRED + l] =
            ((wsum[0][l] + wsum[1][l]) + wsum[2][l]) + wsum[3][l];
    }
}

// Second pass: out[l] = sum over parts of partial[part][l], in a fixed order.
__global__ __launch_bounds__(256) void k_finish(const double *part, int nparts, int nlanes,
                                                double *out)
{
    __shared__ double sh[256];
    for (int l = 0; l < nlanes; ++l) {
        double s = 0.0;
        for (int i = threadIdx.x; i < nparts; i += 256) s += part[(int64_t)i * nlanes + l];
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[l] = sh[0];
        __syncthreads();
    }
}

// Dense float32 -> block-major storage of one species.  Inactive slots get 0 and
// Dirichlet voxels their held value (the highest flagged face wins on shared edges).
template <typename T, int B>
__global__ __launch_bounds__(256) void k_scatter(const BlockInfo *info, const uint64_t *mask,
                                                 const GeomInfo *geom, int nb, const float *dense,
                                                 T *field, uint32_t dir, float d0, float d1,
                                                 float d2, float d3, float d4, float d5)
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
        if (own_bit<B>(rec, slot)) {
            v = dense[((int64_t)gz * g.ny + gy) * g.nx + gx];
            const int onf[6] = {gx == 0, gx == g.nx - 1, gy == 0, gy == g.ny - 1, gz == 0,
                                gz == g.nz - 1};
            for (int f = 0; f < 6; ++f)
                if (((dir >> f) & 1u) && onf[f]) v = dv[f];
        }
        rd_st(field, (int64_t)b * K::NS + slot, v);
    }
}

// Block-major storage -> dense float32 (active voxels only; the caller zero-fills).
template <typename T, int B>
__global__ __launch_bounds__(256) void k_gather(const BlockInfo *info, const uint64_t *mask,
                                                const GeomInfo *geom, int nb, const T *field,
                                                float *dense)
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
        dense[((int64_t)gz * g.ny + gy) * g.nx + gx] = rd_ld(field, (int64_t)b * K::NS + slot);
    }
}

// Set the Dirichlet voxels of one species in a block-major field (others untouched).
template <typename T, int B>
__global__ __launch_bounds__(256) void k_set_dirichlet(const BlockInfo *info, const uint64_t *mask,
                                                       const GeomInfo *geom, int nb, T *field,
                                                       uint32_t dir, float d0, float d1, float d2,
                                                       float d3, float d4, float d5)
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
        if (hit) rd_st(field, (int64_t)b * K::NS + slot, v);
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

template <typename T, int B>
int launch_step_t(const StepArgs &a, hipStream_t st)
{
    int groups = groups_for<B>(a.nb);
    if (a.xcd_chunk > 0) groups = 8 * a.xcd_chunk;
    hipLaunchKernelGGL((k_step<T, B>), dim3(groups), dim3(256), 0, st, a);
    return (int)hipGetLastError();
}

template <typename T, int B>
int launch_reduce_t(const ReduceArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL((k_reduce<T, B>), dim3(groups_for<B>(a.nb)), dim3(256), 0, st, a);
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

int rd_launch_reduce(int storage, int B, const ReduceArgs &a, int, void *stream)
{
    if (a.nb <= 0) return 0;
    RD_DISPATCH(storage, B, launch_reduce_t, a, (hipStream_t)stream);
}

int rd_launch_finish_reduce(const double *partial, int nparts, int nlanes, double *out,
                            void *stream)
{
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, (hipStream_t)stream, partial, nparts,
                       nlanes, out);
    return (int)hipGetLastError();
}

namespace {
template <typename T, int B>
int launch_scatter_t(const BlockInfo *info, const uint64_t *mask, const GeomInfo *geom, int nb,
                     const float *dense, void *field, uint32_t dir, const float *dv, hipStream_t st)
{
    hipLaunchKernelGGL((k_scatter<T, B>), dim3(nb), dim3(256), 0, st, info, mask, geom, nb, dense,
                       (T *)field, dir, dv[0], dv[1], dv[2], dv[3], dv[4], dv[5]);
    return (int)hipGetLastError();
}
template <typename T, int B>
int launch_gather_t(const BlockInfo *info, const uint64_t *mask, const GeomInfo *geom, int nb,
                    const void *field, float *dense, hipStream_t st)
{
    hipLaunchKernelGGL((k_gather<T, B>), dim3(nb), dim3(256), 0, st, info, mask, geom, nb,
                       (const T *)field, dense);
    return (int)hipGetLastError();
}
}  // namespace

int rd_launch_scatter(int storage, int B, const BlockInfo *info, const uint64_t *mask,
                      const GeomInfo *geom, int nb, const float *dense, void *field, uint32_t dir,
                      float dir_value_per_face[6], void *stream)
{
    if (nb <= 0) return 0;
    RD_DISPATCH(storage, B, launch_scatter_t, info, mask, geom, nb, dense, field, dir,
                dir_value_per_face, (hipStream_t)stream);
}

int rd_launch_gather(int storage, int B, const BlockInfo *info, const uint64_t *mask,
                     const GeomInfo *geom, int nb, const void *field, float *dense, int64_t ndense,
                     void *stream)
{
    int rc = rd_launch_fill_u32(dense, 0u, ndense, stream);
    if (rc || nb <= 0) return rc;
    RD_DISPATCH(storage, B, launch_gather_t, info, mask, geom, nb, field, dense,
                (hipStream_t)stream);
}

namespace {
template <typename T, int B>
int launch_setdir_t(const BlockInfo *info, const uint64_t *mask, const GeomInfo *geom, int nb,
                    void *field, uint32_t dir, const float *dv, hipStream_t st)
{
    hipLaunchKernelGGL((k_set_dirichlet<T, B>), dim3(nb), dim3(256), 0, st, info, mask, geom, nb,
                       (T *)field, dir, dv[0], dv[1], dv[2], dv[3], dv[4], dv[5]);
    return (int)hipGetLastError();
}
}  // namespace

int rd_launch_set_dirichlet(int storage, int B, const BlockInfo *info, const uint64_t *mask,
                            const GeomInfo *geom, int nb, void *field, uint32_t dir,
                            const float dv[6], void *stream)
{
    if (nb <= 0) return 0;
    RD_DISPATCH(storage, B, launch_setdir_t, info, mask, geom, nb, field, dir, dv,
                (hipStream_t)stream);
}

int rd_launch_add_u32(uint32_t *ptr, uint32_t add, void *stream)
{
    hipLaunchKernelGGL(k_add_u32, dim3(1), dim3(64), 0, (hipStream_t)stream, ptr, add);
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
