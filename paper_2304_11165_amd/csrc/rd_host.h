// rd_host.h -- host-side objects behind the C ABI handles.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/rd.h"
#include "rd_internal.h"

// Thread-local error detail; returns the status so call sites can `return fail(...)`.
rd_status rd_fail(rd_status s, const std::string &msg);

struct rd_geometry {
    int64_t nx = 0, ny = 0, nz = 0;
    double dx = 1.0;
    int B = 8;
    int64_t NBx = 0, NBy = 0, NBz = 0;
    int64_t n_active = 0;
    std::vector<int64_t> block_id;   // [nb], ascending linear id
    std::vector<BlockInfo> info;     // [nb]
    std::vector<uint64_t> mask;      // [nb * mask_words(B)]
    // per-slot neighbour code [nb * B^3]: bit d (d = 0..5, order -x,+x,-y,+y,-z,+z) set
    // when that face neighbour is an active voxel, bit 6 set when the slot is active
    std::vector<uint8_t> code;
    // Several geometries stepped together (rd_geometry_concat): one entry per part, in list
    // order (box, first block, offset of its box in the dense array that holds the parts'
    // boxes one after another); block_id and the block records' geometry ids refer to the
    // part.  nx holds the dense size and ny = nz = 1 then.  Empty for one geometry.
    std::vector<GeomInfo> parts;
    int nparts() const { return parts.empty() ? 1 : (int)parts.size(); }
    int64_t dense_size() const { return nx * ny * nz; }
    int64_t nb() const { return (int64_t)block_id.size(); }
};

// Builds the index (geometry.cpp).
rd_status rd_geometry_build(const uint8_t *image, int64_t nx, int64_t ny, int64_t nz, int B,
                            rd_geometry *g);
// Compact layout (B = 8): cbase[b] = index of block b's first active voxel when only
// active voxels are stored, in list and slot order (cbase[nb] = active voxels), and the
// neighbour codes of the active voxels in that order.
void rd_geometry_compact_index(const rd_geometry *g, std::vector<uint32_t> &cbase, std::vector<uint8_t> &ccode);
