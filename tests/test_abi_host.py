"""Host-side tests of the C ABI (no GPU): library loads, exports every declared
symbol, builds a bit-exact active-block index, and rejects bad input with the
documented status codes before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def rd():
    from paper_2304_11165_amd import rd as rdmod

    return rdmod


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "rd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(rd_[A-Za-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_every_declared_symbol_is_exported(rd):
    declared = _declared_functions()
    assert len(declared) >= 30
    lib = ctypes.CDLL(rd.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(rd.EXPORTED)


@pytest.mark.parametrize("B", [4, 8])
@pytest.mark.parametrize("seed", range(8))
def test_index_bit_exact_random(rd, oracle_mod, B, seed):
    img = W.random_tiny_geometry(seed, density=[0.01, 0.3, 0.9, None][seed % 4])
    g = rd.Geometry(img, None, 1.0, B)
    ids, nbr = g.export_index()
    masks = g.export_masks()
    i2, n2, m2 = oracle_mod.active_index(img, B)
    np.testing.assert_array_equal(ids, i2)
    np.testing.assert_array_equal(nbr, n2)
    np.testing.assert_array_equal(masks, m2)
    st = g.stats()
    assert st["n_active"] == int(img.astype(bool).sum())
    assert st["n_blocks"] == len(i2)


def _codes_numpy(img, ids, B):
    """Neighbour codes from the image: bit d for an active face neighbour (order
    -x,+x,-y,+y,-z,+z; outside the box = inactive), bit 6 for an active slot."""
    act = np.asarray(img) != 0
    nz, ny, nx = act.shape
    NBx, NBy = -(-nx // B), -(-ny // B)
    pad = np.zeros((nz + 2 + B, ny + 2 + B, nx + 2 + B), dtype=bool)
    pad[1:nz + 1, 1:ny + 1, 1:nx + 1] = act
    out = np.zeros((len(ids), B ** 3), dtype=np.uint8)
    lz, ly, lx = np.meshgrid(np.arange(B), np.arange(B), np.arange(B), indexing="ij")
    lz, ly, lx = lz.ravel(), ly.ravel(), lx.ravel()
    for i, l in enumerate(ids):
        bx, by, bz = l % NBx, (l // NBx) % NBy, l // (NBx * NBy)
        x, y, z = bx * B + lx + 1, by * B + ly + 1, bz * B + lz + 1
        c = np.zeros(B ** 3, dtype=np.uint8)
        for d, (dx, dy, dz) in enumerate([(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0),
                                          (0, 0, -1), (0, 0, 1)]):
            c |= pad[z + dz, y + dy, x + dx].astype(np.uint8) << d
        c |= pad[z, y, x].astype(np.uint8) << 6
        out[i] = c
    return out


@pytest.mark.parametrize("B", [4, 8])
@pytest.mark.parametrize("seed", range(6))
def test_neighbour_codes_bit_exact(rd, oracle_mod, B, seed):
    img = W.random_tiny_geometry(seed, density=[0.05, 0.5, 0.95][seed % 3])
    g = rd.Geometry(img, None, 1.0, B)
    ids, _ = g.export_index()
    np.testing.assert_array_equal(g.export_codes(), _codes_numpy(img, ids, B))


@pytest.mark.parametrize("B", [4, 8])
def test_index_bit_exact_workloads(rd, oracle_mod, B):
    for name in ("spheres64", "decay256"):
        img, sdf = W.workload_geometry(name, small=True)
        g = rd.Geometry(img, sdf, 1.0, B)
        ids, nbr = g.export_index()
        i2, n2, m2 = oracle_mod.active_index(img, B)
        np.testing.assert_array_equal(ids, i2)
        np.testing.assert_array_equal(nbr, n2)
        np.testing.assert_array_equal(g.export_masks(), m2)


def test_index_single_sphere_count(rd):
    img, phi = W.single_sphere(40, (19.5, 20.25, 18.75), 11.0)
    g = rd.Geometry(img, phi, 1.0, 8)
    count = 0
    for z in range(40):
        for y in range(40):
            for x in range(40):
                count += (x - 19.5) ** 2 + (y - 20.25) ** 2 + (z - 18.75) ** 2 > 121.0
    assert g.stats()["n_active"] == count


def test_empty_geometry(rd):
    g = rd.Geometry(np.zeros((5, 6, 7), np.uint8), None, 1.0, 8)
    st = g.stats()
    assert st["n_blocks"] == 0 and st["n_active"] == 0


def test_inconsistent_sdf_rejected(rd):
    img, phi = W.single_sphere(16, (7.5, 7.5, 7.5), 4.0)
    phi = phi.copy()
    phi[3, 4, 5] = -phi[3, 4, 5]
    with pytest.raises(rd.RDError) as e:
        rd.Geometry(img, phi, 1.0, 8)
    assert e.value.name == "RD_ERR_INCONSISTENT_SDF"
    assert "(5,4,3)" in str(e.value)


@pytest.mark.parametrize("shape,B,code", [((0, 4, 4), 8, "RD_ERR_SHAPE"), ((4, 4, 4), 6, "RD_ERR_SHAPE")])
def test_bad_shapes_rejected(rd, shape, B, code):
    with pytest.raises(rd.RDError) as e:
        rd.Geometry(np.ones(shape, np.uint8), None, 1.0, B)
    assert e.value.name == code


def test_bad_dx_rejected(rd):
    with pytest.raises(rd.RDError) as e:
        rd.Geometry(np.ones((4, 4, 4), np.uint8), None, -1.0, 8)
    assert e.value.name == "RD_ERR_ARG"


def test_sim_setup_validation_without_gpu(rd):
    g = rd.Geometry(np.ones((8, 8, 8), np.uint8), None, 1.0, 8)
    s = rd.Sim(g, "fp32")
    with pytest.raises(rd.RDError) as e:
        s.workspace_bytes()
    assert e.value.name == "RD_ERR_STATE"
    assert s.add_species(1.0) == 0
    assert s.add_species(0.4) == 1
    with pytest.raises(rd.RDError):
        s.add_species(-1.0)
    with pytest.raises(rd.RDError):
        s.add_reaction(0, 0, 0.1)
    with pytest.raises(rd.RDError):
        s.add_reaction(0, 5, 0.1)
    s.add_reaction(0, 1, 0.01)
    with pytest.raises(rd.RDError):
        s.set_dirichlet(0, 6, 1.0)
    with pytest.raises(rd.RDError):
        s.set_robin(3, 0.1)
    s.set_dirichlet(0, 0, 1.0)
    # stepping before a workspace is bound is an ordering error, not a crash
    with pytest.raises(rd.RDError) as e:
        s.step(0.1, 1)
    assert e.value.name == "RD_ERR_STATE"
    # workspace size: 2 buffers x 2 species x 512 slots x 4 B at least
    assert s.workspace_bytes() >= 2 * 2 * 512 * 4
    assert s.workspace_bytes(features=1) > s.workspace_bytes()
    assert s.workspace_bytes(features=2, checkpoint_slots=10) > s.workspace_bytes(features=2)
    with pytest.raises(rd.RDError) as e:
        rd._check(rd._lib.rd_sim_bind(s.handle, None, 0, 0, 0, None), "rd_sim_bind")
    assert e.value.name == "RD_ERR_WORKSPACE"


def test_storage_halves_field_bytes(rd):
    g = rd.Geometry(np.ones((16, 16, 16), np.uint8), None, 1.0, 8)
    a, b = rd.Sim(g, "fp32"), rd.Sim(g, "bf16")
    a.add_species(1.0)
    b.add_species(1.0)
    fa, fb = a.workspace_bytes(), b.workspace_bytes()
    assert fa - fb == 2 * 8 * 512 * 2  # two buffers, 8 blocks, 2 bytes saved per slot


def test_status_strings(rd):
    for i, name in enumerate(rd.STATUS):
        assert rd._lib.rd_status_string(i).decode()


def test_new_entry_points_validate_without_gpu(rd):
    """Argument and ordering checks of the diffusivity, sink, FRAP and distance-transform
    entry points run on the host and fail cleanly before any GPU work."""
    import ctypes

    g = rd.Geometry(np.ones((8, 8, 8), np.uint8), None, 1.0, 8)
    s = rd.Sim(g, "fp32")
    s.add_species(1.0)
    base = s.workspace_bytes()
    # the factor adds 4 bytes per slot (+ counters); with the adjoint, dL/de adds 8
    assert s.workspace_bytes(features=rd.RD_WS_DIFFUSIVITY) >= base + 4 * 512
    assert (s.workspace_bytes(features=rd.RD_WS_DIFFUSIVITY | rd.RD_WS_ADJOINT, checkpoint_slots=4) -
            s.workspace_bytes(features=rd.RD_WS_ADJOINT, checkpoint_slots=4)) >= 12 * 512
    with pytest.raises(rd.RDError) as e:
        s.set_sink(0, -1.0)
    assert e.value.name == "RD_ERR_ARG"
    with pytest.raises(rd.RDError) as e:
        s.set_sink(2, 0.1)
    assert e.value.name == "RD_ERR_ARG"
    s.set_sink(0, 0.1)
    P = ctypes.c_void_p
    for call in (lambda: rd._lib.rd_sim_set_diffusivity(s.handle, P(8)),
                 lambda: rd._lib.rd_sim_set_sink_band(s.handle, P(8), ctypes.c_double(1.0), None),
                 lambda: rd._lib.rd_sim_region_mass(s.handle, 0, P(8), P(8))):
        with pytest.raises(rd.RDError) as e:
            rd._check(call(), "call before bind")
        assert e.value.name == "RD_ERR_STATE"
    n = ctypes.c_size_t()
    rd._check(rd._lib.rd_sdf_scratch_bytes(10, 20, 30, ctypes.byref(n)), "rd_sdf_scratch_bytes")
    assert n.value >= 20 * 10 * 20 * 30
    with pytest.raises(rd.RDError) as e:
        rd._check(rd._lib.rd_sdf_scratch_bytes(0, 20, 30, ctypes.byref(n)), "rd_sdf_scratch_bytes")
    assert e.value.name == "RD_ERR_SHAPE"
    with pytest.raises(rd.RDError) as e:  # NULL pointers are refused before any launch
        rd._check(rd._lib.rd_sdf_from_image(None, 4, 4, 4, ctypes.c_double(1.0), None, None, 0, None),
                  "rd_sdf_from_image")
    assert e.value.name == "RD_ERR_ARG"


def test_compact_layout_validation_without_gpu(rd):
    img, _ = W.boolean_spheres(40, 0.4, 2.0, 5.0, seed=3)
    g8 = rd.Geometry(img, None, 1.0, 8)
    blocks, compact = rd.Sim(g8, "fp32"), rd.Sim(g8, "fp32")
    for s in (blocks, compact):
        s.add_species(1.0)
        s.add_species(0.5)
    with pytest.raises(rd.RDError) as e:
        rd._check(rd._lib.rd_sim_set_layout(compact.handle, 2), "rd_sim_set_layout")
    assert e.value.name == "RD_ERR_ARG"
    compact.set_layout("compact")
    # the block kernels do not exist for the compact layout
    with pytest.raises(rd.RDError) as e:
        compact.set_kernel("block")
    assert e.value.name == "RD_ERR_STATE"
    compact.set_kernel("column_xch")
    # the fields shrink from whole blocks to the active voxels (2 buffers x 2 species x 4 B)
    st = g8.stats()
    saved = blocks.workspace_bytes() - compact.workspace_bytes()
    slots = st["n_blocks"] * 512
    assert saved >= 2 * 2 * 4 * (slots - st["n_active"]) - 2 * 2 * 4 * 64 - 4096
    assert saved > 0
    # 4^3 blocks have no compact form
    g4 = rd.Geometry(img, None, 1.0, 4)
    s4 = rd.Sim(g4, "fp32")
    s4.add_species(1.0)
    with pytest.raises(rd.RDError) as e:
        s4.set_layout("compact")
    assert e.value.name == "RD_ERR_SHAPE"


def test_concat_geometry_structure(rd):
    """rd_geometry_concat: the parts' block lists one after another, neighbour indices
    shifted by the part's first block, masks and codes unchanged, boxes one after another
    in the dense array; mixed block edges, nested concatenations and batches of
    concatenations are refused."""
    rng = np.random.default_rng(4)
    imgs = [(rng.random(s) < p).astype(np.uint8) for s, p in
            (((20, 17, 23), 0.6), ((9, 30, 11), 0.5), ((5, 5, 5), 0.0), ((13, 8, 21), 0.7))]
    for B in (4, 8):
        gs = [rd.Geometry(img, None, 1.0, B) for img in imgs]
        cat = rd.Geometry.concat(gs)
        parts = cat.parts()
        ids, nbr = cat.export_index()
        masks, codes = cat.export_masks(), cat.export_codes()
        off = dense = 0
        for g, img, p in zip(gs, imgs, parts):
            i1, n1 = g.export_index()
            nb = len(i1)
            assert p == {"shape": img.shape, "dense_offset": dense, "first_block": off, "n_blocks": nb}
            assert np.array_equal(ids[off:off + nb], i1)
            assert np.array_equal(nbr[off:off + nb], np.where(n1 >= 0, n1 + off, -1))
            assert np.array_equal(masks[off:off + nb], g.export_masks())
            assert np.array_equal(codes[off:off + nb], g.export_codes())
            off += nb
            dense += img.size
        st = cat.stats()
        assert st["n_blocks"] == off and cat.shape == (1, 1, dense)
        assert st["n_active"] == sum(int(img.sum()) for img in imgs)
        # a plain geometry is one part
        assert gs[0].parts() == [{"shape": imgs[0].shape, "dense_offset": 0, "first_block": 0,
                                  "n_blocks": gs[0].stats()["n_blocks"]}]
        with pytest.raises(rd.RDError) as e:
            rd.Geometry.concat([cat, gs[0]])
        assert e.value.name == "RD_ERR_ARG"
        with pytest.raises(rd.RDError) as e:
            rd.Batch([cat])
        assert e.value.name == "RD_ERR_ARG"
    g4, g8 = rd.Geometry(imgs[0], None, 1.0, 4), rd.Geometry(imgs[0], None, 1.0, 8)
    with pytest.raises(rd.RDError) as e:
        rd.Geometry.concat([g4, g8])
    assert e.value.name == "RD_ERR_SHAPE"
    with pytest.raises(rd.RDError) as e:
        rd._check(rd._lib.rd_geometry_part_info(g8.handle, 1, None, None, None, None), "rd_geometry_part_info")
    assert e.value.name == "RD_ERR_ARG"


def test_fused_steps_validation_without_gpu(rd):
    img, _ = W.boolean_spheres(40, 0.4, 2.0, 5.0, seed=3)
    s8 = rd.Sim(rd.Geometry(img, None, 1.0, 8), "fp32")
    s8.add_species(1.0)
    assert s8.get_fused_steps() == 1
    s8.set_fused_steps(16)
    assert s8.get_fused_steps() == 16
    for bad in (0, 257):
        with pytest.raises(rd.RDError) as e:
            s8.set_fused_steps(bad)
        assert e.value.name == "RD_ERR_ARG"
    s4 = rd.Sim(rd.Geometry(img, None, 1.0, 4), "fp32")
    s4.add_species(1.0)
    with pytest.raises(rd.RDError) as e:
        s4.set_fused_steps(4)
    assert e.value.name == "RD_ERR_STATE"
    sc = rd.Sim(rd.Geometry(img, None, 1.0, 8), "fp32")
    sc.add_species(1.0)
    sc.set_layout("compact")
    with pytest.raises(rd.RDError) as e:
        sc.set_fused_steps(4)
    assert e.value.name == "RD_ERR_STATE"
