// k_edt.hip -- signed distance of a voxel image on the GPU (exact Euclidean distance
// transform), the level-set description of the pore space (paper: section "Level-set
// method for image-based geometry reconstruction", eq. SDF; building it on the GPU is
// the future work named in section "Discussion and conclusions").
//
// phi at an active voxel is (distance to the nearest inactive voxel centre - 1/2) dx, at
// an inactive voxel -(distance to the nearest active voxel centre - 1/2) dx; with no
// voxel of the other phase it is +-(box diagonal) dx.  Squared distances are exact
// integers (uint32) from the separable lower-envelope-of-parabolas transform of
// Felzenszwalb and Huttenlocher ("Distance transforms of sampled functions", Theory of
// Computing 8, 2012): a scan along x gives the squared distance to the nearest feature
// of the row, then each line along y and along z is replaced by
// min_k ((j - k)^2 + f(k)).  One wave per row for the scan, one thread per line for the
// envelope passes; the envelope's vertices, heights and
// interval boundaries live in a global scratch interleaved by line, so that
// neighbouring threads touch neighbouring words.  HBM-bound: a few bytes per voxel and
// pass, no arithmetic to speak of.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>
#include <string>

#include "rd_host.h"

namespace {

constexpr uint32_t EDT_INF = 0xffffffffu;

// Pass along x: g = squared distance to the nearest feature voxel of the row
// (EDT_INF if the row has none).  feature_inactive = 1: inactive voxels are features.
// One wave per row, 64 consecutive voxels per step: the nearest feature to the left is
// a running prefix maximum of feature indices across the lanes (carried from chunk to
// chunk), the nearest to the right a suffix minimum taken from the far end.
__global__ __launch_bounds__(256) void k_edt_x(const uint8_t *__restrict__ img, int nx, int64_t nrows,
                                               int feature_inactive, uint32_t *__restrict__ g)
{
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= nrows) return;  // whole waves
    const uint8_t *r = img + row * nx;
    uint32_t *out = g + row * nx;
    int carry = -1;
    for (int c0 = 0; c0 < nx; c0 += 64) {
        const int i = c0 + lane;
        const bool f = i < nx && ((r[i] == 0) == (feature_inactive != 0));
        int v = f ? i : -1;
        for (int o = 1; o < 64; o <<= 1) {
            const int u = __shfl_up(v, o, 64);
            if (lane >= o) v = max(v, u);
        }
        v = max(v, carry);
        carry = __shfl(v, 63, 64);
        if (i < nx) out[i] = v < 0 ? EDT_INF : (uint32_t)(i - v);
    }
    int carry2 = 0x7fffffff;
    for (int c0 = ((nx - 1) / 64) * 64; c0 >= 0; c0 -= 64) {
        const int i = c0 + lane;
        const bool f = i < nx && ((r[i] == 0) == (feature_inactive != 0));
        int v = f ? i : 0x7fffffff;
        for (int o = 1; o < 64; o <<= 1) {
            const int u = __shfl_down(v, o, 64);
            if (lane + o < 64) v = min(v, u);
        }
        v = min(v, carry2);
        carry2 = __shfl(v, 0, 64);
        if (i < nx) {
            uint32_t d = out[i];
            if (v != 0x7fffffff && (uint32_t)(v - i) < d) d = (uint32_t)(v - i);
            out[i] = d == EDT_INF ? EDT_INF : d * d;
        }
    }
}

// One line of n samples of g, at stride st from base, replaced by its distance
// transform min_k ((j - k)^2 + g(k)).  Line `line` of `nl` lines owns the scratch words
// V[k * nl + line] (vertex), H[...] (its height g(vertex)), Z[...] (left end of its
// interval).  The top of the envelope is held in registers and written through, so the
// scratch is read back only when a parabola is dropped or the evaluation moves on.
__global__ __launch_bounds__(256) void k_edt_lines(uint32_t *__restrict__ g, int n, int64_t st, int64_t nl,
                                                   int lines_x, int64_t lstride_x, int64_t lstride_y,
                                                   int32_t *__restrict__ V, uint32_t *__restrict__ H,
                                                   double *__restrict__ Z)
{
    const int64_t line = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (line >= nl) return;
    const int64_t base = (line % lines_x) * lstride_x + (line / lines_x) * lstride_y;
    int kk = -1;  // top of the envelope
    int tv = 0;   // its vertex, height and left end
    uint32_t th = 0;
    double tz = -INFINITY;
    for (int q = 0; q < n; ++q) {
        const uint32_t fq = g[base + q * st];
        if (fq == EDT_INF) continue;
        const double hq = (double)fq + (double)q * (double)q;  // exact: below 2^53
        double s = -INFINITY;
        while (kk >= 0) {
            const double hp = (double)th + (double)tv * (double)tv;
            s = (hq - hp) / (2.0 * (double)(q - tv));  // where the two parabolas cross
            if (s > tz) break;
            --kk;  // the top parabola is nowhere lowest: drop it
            s = -INFINITY;
            if (kk >= 0) {
                tv = V[(int64_t)kk * nl + line];
                th = H[(int64_t)kk * nl + line];
                tz = Z[(int64_t)kk * nl + line];
            }
        }
        ++kk;
        tv = q;
        th = fq;
        tz = s;
        V[(int64_t)kk * nl + line] = q;
        H[(int64_t)kk * nl + line] = fq;
        Z[(int64_t)kk * nl + line] = s;
    }
    if (kk < 0) return;  // no finite sample: the line stays EDT_INF
    int k = 0;
    int cv = V[line];
    uint32_t ch = H[line];
    double nzb = kk >= 1 ? Z[nl + line] : INFINITY;  // left end of the next interval
    for (int j = 0; j < n; ++j) {
        while (nzb < (double)j) {
            ++k;
            cv = V[(int64_t)k * nl + line];
            ch = H[(int64_t)k * nl + line];
            nzb = k < kk ? Z[(int64_t)(k + 1) * nl + line] : INFINITY;
        }
        const int64_t d = (int64_t)j - cv;
        g[base + j * st] = (uint32_t)(d * d + (int64_t)ch);
    }
}

// phi of the voxels of one phase from the squared distances to the other phase.
__global__ __launch_bounds__(256) void k_edt_finish(const uint8_t *img, const uint32_t *g, int64_t n, int active,
                                                    double dx, double diag, float *sdf)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    if ((img[i] != 0) != (active != 0)) return;
    const double d = g[i] == EDT_INF ? diag : sqrt((double)g[i]) - 0.5;
    sdf[i] = (float)((active ? d : -d) * dx);
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Fixed scratch of rd_sdf_from_image_static: one array per GPU, resident until the
// process ends.  Host code uses only the device address fetched per device below; the
// array's name on the host is a stand-in, not a device address.
#define RD_SDF_STATIC_BYTES ((size_t)64 << 20)
static __device__ __align__(256) unsigned char scratch[RD_SDF_STATIC_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex static_mu;
void *static_ptr[MAX_DEVICES];  // device address of `scratch` on each device, or NULL
}  // namespace

extern "C" rd_status rd_sdf_scratch_bytes(int64_t nx, int64_t ny, int64_t nz, size_t *bytes)
{
    if (!bytes) return rd_fail(RD_ERR_ARG, "bytes is NULL");
    if (nx < 1 || ny < 1 || nz < 1) return rd_fail(RD_ERR_SHAPE, "need nx, ny, nz >= 1");
    const size_t N = (size_t)nx * (size_t)ny * (size_t)nz;
    *bytes = align256(4 * N) + align256(4 * N) + align256(4 * N) + align256(8 * N);
    return RD_OK;
}

extern "C" rd_status rd_sdf_from_image_static(const uint8_t *dev_image, int64_t nx, int64_t ny, int64_t nz,
                                              double dx, float *dev_sdf, void *stream)
{
    if (!dev_image || !dev_sdf) return rd_fail(RD_ERR_ARG, "NULL pointer");
    if (nx < 1 || ny < 1 || nz < 1 || nx > 32768 || ny > 32768 || nz > 32768)
        return rd_fail(RD_ERR_SHAPE, "need 1 <= nx, ny, nz <= 32768");
    size_t need = 0;
    rd_sdf_scratch_bytes(nx, ny, nz, &need);
    if (need > RD_SDF_STATIC_BYTES)
        return rd_fail(RD_ERR_SHAPE, "volume needs " + std::to_string(need) + " scratch bytes; the fixed scratch holds " +
                                         std::to_string(RD_SDF_STATIC_BYTES) + " (20 bytes per voxel)");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return rd_fail(RD_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= MAX_DEVICES) return rd_fail(RD_ERR_HIP, "device id out of range");
    void *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lock(static_mu);
        if (!static_ptr[dev]) {  // first call on this device (it is current)
            e = hipGetSymbolAddress(&static_ptr[dev], HIP_SYMBOL(scratch));
            if (e != hipSuccess) {
                static_ptr[dev] = nullptr;
                return rd_fail(RD_ERR_HIP, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
            }
        }
        ptr = static_ptr[dev];
    }
    return rd_sdf_from_image(dev_image, nx, ny, nz, dx, dev_sdf, ptr, RD_SDF_STATIC_BYTES, stream);
}

extern "C" rd_status rd_sdf_from_image(const uint8_t *dev_image, int64_t nx, int64_t ny, int64_t nz, double dx,
                                       float *dev_sdf, void *dev_scratch, size_t scratch_bytes, void *stream)
{
    if (!dev_image || !dev_sdf || !dev_scratch) return rd_fail(RD_ERR_ARG, "NULL pointer");
    if (!(dx > 0.0)) return rd_fail(RD_ERR_ARG, "dx must be > 0");
    if (nx < 1 || ny < 1 || nz < 1 || nx > 32768 || ny > 32768 || nz > 32768)
        return rd_fail(RD_ERR_SHAPE, "need 1 <= nx, ny, nz <= 32768");
    size_t need = 0;
    rd_sdf_scratch_bytes(nx, ny, nz, &need);
    if (scratch_bytes < need)
        return rd_fail(RD_ERR_WORKSPACE, "scratch has " + std::to_string(scratch_bytes) + " bytes, needs " +
                                             std::to_string(need));
    const int64_t N = nx * ny * nz;
    char *p = (char *)dev_scratch;
    uint32_t *g = (uint32_t *)p;
    int32_t *V = (int32_t *)(p + align256(4 * (size_t)N));
    uint32_t *H = (uint32_t *)(p + 2 * align256(4 * (size_t)N));
    double *Z = (double *)(p + 3 * align256(4 * (size_t)N));
    hipStream_t st = (hipStream_t)stream;
    const double diag = sqrt((double)nx * nx + (double)ny * ny + (double)nz * nz);
    for (int active = 1; active >= 0; --active) {
        // features: the other phase
        hipLaunchKernelGGL(k_edt_x, dim3((unsigned)((ny * nz + 3) / 4)), dim3(256), 0, st, dev_image, (int)nx,
                           ny * nz, active, g);
        // lines along y: line = x + nx z, base = x + nx ny z, stride nx
        hipLaunchKernelGGL(k_edt_lines, dim3(blocks_for(nx * nz)), dim3(256), 0, st, g, (int)ny, nx, nx * nz,
                           (int)nx, (int64_t)1, nx * ny, V, H, Z);
        // lines along z: line = x + nx y, base = x + nx y, stride nx ny
        hipLaunchKernelGGL(k_edt_lines, dim3(blocks_for(nx * ny)), dim3(256), 0, st, g, (int)nz, nx * ny, nx * ny,
                           (int)nx, (int64_t)1, nx, V, H, Z);
        hipLaunchKernelGGL(k_edt_finish, dim3(blocks_for(N)), dim3(256), 0, st, dev_image, g, N, active, dx, diag,
                           dev_sdf);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return rd_fail(RD_ERR_HIP, std::string("EDT launch: ") + hipGetErrorString(e));
    return RD_OK;
}
