// k_frap.hip -- FP64 mass of a field inside an axis-aligned box of voxels, for the
// bleached region of a simulated FRAP experiment (paper: section "Calculation of
// effective diffusion coefficient and tortuosity").  HBM-bound; blocks that do not
// meet the box are skipped without reading the field.
#include "rd_device.h"
#include "rd_frap.h"

namespace {

struct Region {
    int32_t lo[3], hi[3];  // x, y, z: lo <= g < hi
};

// B = 8: one block per workgroup, two slots per thread; B = 4: four blocks per
// workgroup, one slot per thread.  One partial per workgroup: the wave sums in order.
// cbase: compact layout (B = 8; only active voxels stored) or NULL (block-major).
template <typename T, int B>
__global__ __launch_bounds__(256) void k_region_mass(const BlockInfo *info, const uint8_t *code,
                                                     const uint32_t *cbase, const uint64_t *mask, const T *c,
                                                     int nb, Region r, double *partial)
{
    using C = Cfg<B>;
    constexpr int NS = B * B * B;
    __shared__ double wsum[4];
    const int sub = threadIdx.x / C::TPB, lt = threadIdx.x % C::TPB;
    const int b = blockIdx.x * C::BPW + sub;
    double acc = 0.0;
    if (b < nb) {
        int bx, by, bz, gid;
        block_pos(info[b], &bx, &by, &bz, &gid);
        const int o[3] = {bx * B, by * B, bz * B};
        bool meets = true;
        for (int d = 0; d < 3; ++d) meets = meets && o[d] < r.hi[d] && o[d] + B > r.lo[d];
        if (meets) {
            for (int k = 0; k < C::VPT; ++k) {
                const int slot = lt + k * C::TPB;
                const int g[3] = {o[0] + slot % B, o[1] + (slot / B) % B, o[2] + slot / (B * B)};
                bool in = true;
                for (int d = 0; d < 3; ++d) in = in && g[d] >= r.lo[d] && g[d] < r.hi[d];
                if (cbase) in = in && own_bit<B>(mask + (int64_t)b * Blk<B>::MW, slot);
                if (!in) continue;
                const int64_t i = cbase ? slot_index8(cbase, mask, b, slot) : (int64_t)b * NS + slot;
                if (code[i] & 64u) acc += (double)rd_ld(c, i);
            }
        }
    }
    const double v = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
}

template <typename T>
void launch_t(int B, const BlockInfo *info, const uint8_t *code, const uint32_t *cbase, const uint64_t *mask,
              const void *c, int nb, Region r, double *partial, hipStream_t st)
{
    const dim3 grid((unsigned)rd_region_rows(B, nb));
    if (B == 8)
        hipLaunchKernelGGL((k_region_mass<T, 8>), grid, dim3(256), 0, st, info, code, cbase, mask, (const T *)c, nb,
                           r, partial);
    else
        hipLaunchKernelGGL((k_region_mass<T, 4>), grid, dim3(256), 0, st, info, code, cbase, mask, (const T *)c, nb,
                           r, partial);
}

}  // namespace

int rd_region_rows(int B, int nb) { return B == 8 ? nb : (nb + 3) / 4; }

int rd_launch_region_mass(int storage, int B, const BlockInfo *info, const uint8_t *code, const uint32_t *cbase,
                          const uint64_t *mask, const void *c, int nb, const int32_t region[6], double *partial,
                          void *stream)
{
    if (nb <= 0) return 0;
    Region r;
    for (int d = 0; d < 3; ++d) {
        r.lo[d] = region[2 * d];
        r.hi[d] = region[2 * d + 1];
    }
    hipStream_t st = (hipStream_t)stream;
    if (storage == 0) launch_t<float>(B, info, code, cbase, mask, c, nb, r, partial, st);
    else if (storage == 1) launch_t<bf16_t>(B, info, code, cbase, mask, c, nb, r, partial, st);
    else launch_t<_Float16>(B, info, code, cbase, mask, c, nb, r, partial, st);
    return (int)hipGetLastError();
}
