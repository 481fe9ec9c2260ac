// geometry.cpp -- host construction of the active-block index.
//
// The paper stores a chunk of B^3 grid points only if it holds at least one point
// of the diffusion phase, and caches the chunk position with an allocation mask
// (section "Parallel implementation using OpenFPM"; section "Generating
// real-world geometries": points with phi > 0 are inserted).  Here that becomes:
//   1. one pass over the image marks occupied blocks and sets their slot bits;
//   2. occupied blocks are numbered in ascending linear id
//      l = (bz*NBy + by)*NBx + bx, which keeps +-x neighbours adjacent in the list
//      and +-y / +-z neighbours at a fixed stride for dense regions;
//   3. a dense block map (linear id -> list index or -1) gives the six face
//      neighbours of every block;
//   4. the face bits of every neighbour are copied next to the block's own bits,
//      so a kernel reads one contiguous mask record per block.
#include <string.h>

#include <algorithm>

#include "rd_host.h"

namespace {

inline int face_bit(int f, int B, int lx, int ly, int lz)
{
    if (f < 2) return lz * B + ly;
    if (f < 4) return lz * B + lx;
    return ly * B + lx;
}

inline bool own_bit(const uint64_t *rec, int B, int slot)
{
    if (B == 8) return (rec[slot >> 6] >> (slot & 63)) & 1u;
    return (rec[0] >> slot) & 1u;
}

inline void set_face_bit(uint64_t *rec, int B, int f, int bit)
{
    if (B == 8) {
        rec[8 + f] |= (uint64_t)1 << bit;
    } else {
        int w = f < 4 ? 1 : 2;
        int sh = f < 4 ? 16 * f : 16 * (f - 4);
        rec[w] |= (uint64_t)1 << (sh + bit);
    }
}

}  // namespace

rd_status rd_geometry_build(const uint8_t *image, int64_t nx, int64_t ny, int64_t nz, int B,
                            rd_geometry *g)
{
    g->nx = nx;
    g->ny = ny;
    g->nz = nz;
    g->B = B;
    g->NBx = (nx + B - 1) / B;
    g->NBy = (ny + B - 1) / B;
    g->NBz = (nz + B - 1) / B;
    if (g->NBx > 65535 || g->NBy > 65535 || g->NBz > 65535)
        return rd_fail(RD_ERR_SHAPE, "more than 65535 blocks along an axis");
    const int64_t nblk = g->NBx * g->NBy * g->NBz;
    const int MW = mask_words(B);
    const int bpw = B == 8 ? 8 : 1;  // own words

    // pass 1: occupancy + own bits in a dense temporary keyed by linear block id
    std::vector<int32_t> map(nblk, -1);
    std::vector<uint64_t> dense_bits;  // grown per newly seen block
    std::vector<int64_t> seen;         // linear ids in order of first sight
    int64_t n_active = 0;
    for (int64_t z = 0; z < nz; ++z) {
        const int64_t bz = z / B, lz = z % B;
        for (int64_t y = 0; y < ny; ++y) {
            const int64_t by = y / B, ly = y % B;
            const uint8_t *row = image + (z * ny + y) * nx;
            for (int64_t x = 0; x < nx; ++x) {
                if (!row[x]) continue;
                const int64_t bx = x / B, lx = x % B;
                const int64_t l = (bz * g->NBy + by) * g->NBx + bx;
                int32_t t = map[l];
                if (t < 0) {
                    t = (int32_t)seen.size();
                    if (seen.size() >= (size_t)INT32_MAX)
                        return rd_fail(RD_ERR_SHAPE, "too many active blocks");
                    map[l] = t;
                    seen.push_back(l);
                    dense_bits.resize(dense_bits.size() + bpw, 0);
                }
                const int slot = (int)((lz * B + ly) * B + lx);
                dense_bits[(size_t)t * bpw + (slot >> 6)] |= (uint64_t)1 << (slot & 63);
                ++n_active;
            }
        }
    }
    g->n_active = n_active;

    // pass 2: ascending linear id
    std::vector<int32_t> by_seen(seen.size());
    {
        std::vector<int32_t> order(seen.size());
        for (size_t i = 0; i < seen.size(); ++i) order[i] = (int32_t)i;
        std::sort(order.begin(), order.end(),
                  [&](int32_t a, int32_t b) { return seen[a] < seen[b]; });
        g->block_id.resize(seen.size());
        for (size_t r = 0; r < order.size(); ++r) {
            g->block_id[r] = seen[order[r]];
            by_seen[order[r]] = (int32_t)r;
        }
        for (size_t i = 0; i < seen.size(); ++i) map[seen[i]] = by_seen[i];
    }
    const int64_t nb = g->nb();

    // own bits in list order
    g->mask.assign((size_t)nb * MW, 0);
    for (size_t i = 0; i < seen.size(); ++i) {
        uint64_t *rec = &g->mask[(size_t)by_seen[i] * MW];
        for (int w = 0; w < bpw; ++w) rec[w] = dense_bits[i * bpw + w];
    }

    // pass 3: neighbours + positions
    static const int DX[6] = {-1, 1, 0, 0, 0, 0}, DY[6] = {0, 0, -1, 1, 0, 0},
                     DZ[6] = {0, 0, 0, 0, -1, 1};
    g->info.resize(nb);
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t l = g->block_id[b];
        const int64_t bx = l % g->NBx, by = (l / g->NBx) % g->NBy, bz = l / (g->NBx * g->NBy);
        BlockInfo &bi = g->info[b];
        for (int f = 0; f < 6; ++f) {
            const int64_t x2 = bx + DX[f], y2 = by + DY[f], z2 = bz + DZ[f];
            int32_t r = -1;
            if (x2 >= 0 && x2 < g->NBx && y2 >= 0 && y2 < g->NBy && z2 >= 0 && z2 < g->NBz)
                r = map[(z2 * g->NBy + y2) * g->NBx + x2];
            bi.nbr[f] = r;
        }
        bi.xy = (int32_t)(bx | (by << 16));
        bi.zg = (int32_t)bz;
    }

    // pass 5 (after the face bits below): per-slot neighbour codes
    struct CodeFill {
        static void run(rd_geometry *g)
        {
            const int B = g->B, NS = B * B * B, MW = mask_words(B);
            const int64_t nb = g->nb();
            g->code.assign((size_t)nb * NS, 0);
            for (int64_t b = 0; b < nb; ++b) {
                const uint64_t *rec = &g->mask[(size_t)b * MW];
                auto own = [&](int s) { return own_bit(rec, B, s); };
                auto face = [&](int f, int bit) {
                    if (B == 8) return (bool)((rec[8 + f] >> bit) & 1u);
                    const int w = f < 4 ? 1 : 2, sh = f < 4 ? 16 * f : 16 * (f - 4);
                    return (bool)((rec[w] >> (sh + bit)) & 1u);
                };
                for (int s = 0; s < NS; ++s) {
                    const int lx = s % B, ly = (s / B) % B, lz = s / (B * B);
                    uint8_t c = 0;
                    if (lx > 0 ? own(s - 1) : face(0, lz * B + ly)) c |= 1;
                    if (lx < B - 1 ? own(s + 1) : face(1, lz * B + ly)) c |= 2;
                    if (ly > 0 ? own(s - B) : face(2, lz * B + lx)) c |= 4;
                    if (ly < B - 1 ? own(s + B) : face(3, lz * B + lx)) c |= 8;
                    if (lz > 0 ? own(s - B * B) : face(4, ly * B + lx)) c |= 16;
                    if (lz < B - 1 ? own(s + B * B) : face(5, ly * B + lx)) c |= 32;
                    if (own(s)) c |= 64;
                    g->code[(size_t)b * NS + s] = c;
                }
            }
        }
    };

    // pass 4: face bits = own bits of the neighbour voxel across each face
    for (int64_t b = 0; b < nb; ++b) {
        uint64_t *rec = &g->mask[(size_t)b * MW];
        for (int f = 0; f < 6; ++f) {
            const int32_t n = g->info[b].nbr[f];
            if (n < 0) continue;
            const uint64_t *nrec = &g->mask[(size_t)n * MW];
            for (int v = 0; v < B; ++v)
                for (int u = 0; u < B; ++u) {
                    int lx, ly, lz;  // position in *this* block's face coordinates
                    int nx_, ny_, nz_;  // the neighbour voxel in the neighbour block
                    if (f < 2) { ly = u; lz = v; lx = f == 0 ? 0 : B - 1; nx_ = f == 0 ? B - 1 : 0; ny_ = ly; nz_ = lz; }
                    else if (f < 4) { lx = u; lz = v; ly = f == 2 ? 0 : B - 1; nx_ = lx; ny_ = f == 2 ? B - 1 : 0; nz_ = lz; }
                    else { lx = u; ly = v; lz = f == 4 ? 0 : B - 1; nx_ = lx; ny_ = ly; nz_ = f == 4 ? B - 1 : 0; }
                    const int nslot = (nz_ * B + ny_) * B + nx_;
                    if (own_bit(nrec, B, nslot)) set_face_bit(rec, B, f, face_bit(f, B, lx, ly, lz));
                }
        }
    }
    // B = 8: words 14-15 of a record hold the number of active slots below each plane
    // (16 bits per plane z = 0..7, plane z at bit 16 (z % 4) of word 14 + z / 4), the
    // offset of the plane's first voxel in the compact layout, where a block stores
    // only its active voxels in slot order
    if (B == 8) {
        for (int64_t b = 0; b < nb; ++b) {
            uint64_t *rec = &g->mask[(size_t)b * MW];
            uint64_t pre = 0;
            rec[14] = rec[15] = 0;
            for (int z = 0; z < 8; ++z) {
                rec[14 + z / 4] |= pre << (16 * (z % 4));
                pre += (uint64_t)__builtin_popcountll(rec[z]);
            }
        }
    }
    CodeFill::run(g);
    return RD_OK;
}

void rd_geometry_compact_index(const rd_geometry *g, std::vector<uint32_t> &cbase, std::vector<uint8_t> &ccode)
{
    const int B = g->B, NS = B * B * B;
    const int64_t nb = g->nb();
    cbase.assign((size_t)nb + 1, 0);
    ccode.clear();
    ccode.reserve((size_t)g->n_active);
    for (int64_t b = 0; b < nb; ++b) {
        cbase[b] = (uint32_t)ccode.size();
        const uint8_t *cd = &g->code[(size_t)b * NS];
        for (int s = 0; s < NS; ++s)
            if (cd[s] & 64u) ccode.push_back(cd[s]);
    }
    cbase[nb] = (uint32_t)ccode.size();
}
