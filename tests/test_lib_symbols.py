"""The C-ABI library loads without a GPU and exports every function include/ogvdb.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ogvdb.h")
LIB = os.path.join(ROOT, "paper_2404_10272_amd", "libogvdb.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ogv_[a-z_]+)\s*\(", text)))


def test_header_declares_the_sampler_boundary():
    names = declared()
    for n in ["ogv_vdb_build", "ogv_dense_build", "ogv_sample_count", "ogv_sample_fill", "ogv_sample_rays",
              "ogv_composite_fwd", "ogv_composite_bwd", "ogv_last_error"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_signatures_cover_header():
    from paper_2404_10272_amd import api
    assert set(declared()) <= set(api.SIGNATURES), set(declared()) - set(api.SIGNATURES)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_side_validation_without_gpu():
    # argument checks run before any device work, so they answer on a CPU host
    from paper_2404_10272_amd import api
    L = api.lib()
    n = ctypes.c_size_t()
    bad = api.make_step("cone", cone=1 / 256, dt_min=1e-3)
    assert L.ogv_sample_workspace_size(-1, 0.0, 1.0, ctypes.byref(bad), ctypes.byref(n)) == -1
    assert L.ogv_sample_workspace_size(100, 0.05, 1000.0, ctypes.byref(bad), ctypes.byref(n)) == 0
    assert n.value > 100 * 4
    h = ctypes.c_void_p()
    boxes = (ctypes.c_float * 6)(0, 0, 0, 1, 1, 1)
    assert L.ogv_vdb_build(1, 0, boxes, ctypes.c_void_p(1), 4, ctypes.byref(h), None) == -1
    assert b"res" in L.ogv_last_error()
    nested_wrong = (ctypes.c_float * 12)(-2, -2, -2, 2, 2, 2, -1, -1, -1, 1, 1, 1)
    assert L.ogv_dense_build(2, 8, nested_wrong, ctypes.c_void_p(1), ctypes.byref(h), None) == -1
    assert b"contain" in L.ogv_last_error()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_scan_entry_validates_on_host():
    # ogv_sample_scan locates the counts from n_rays alone; it refuses a
    # workspace smaller than the count call's prefix, null offsets and bad n
    from paper_2404_10272_amd import api
    L = api.lib()
    n = ctypes.c_size_t()
    unit = api.make_step("const", dt=5e-3)
    assert L.ogv_sample_workspace_size(1000, 2.0, 6.0, ctypes.byref(unit), ctypes.byref(n)) == 0
    fake = ctypes.c_void_p(1 << 20)   # never dereferenced: every call below fails its host checks
    assert L.ogv_sample_scan(-1, fake, fake, n.value, None) == -1
    assert L.ogv_sample_scan(1000, None, fake, n.value, None) == -1
    assert L.ogv_sample_scan(1000, fake, None, n.value, None) == -2
    assert L.ogv_sample_scan(1000, fake, fake, 64, None) == -2
    assert b"workspace" in L.ogv_last_error()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_render_blobs_validates_the_field_on_host():
    from paper_2404_10272_amd import api
    lib = api.lib()
    good = api.blob_field([[0, 0, 0]], [0.5], [1.0], [[1, 1, 1]])
    assert lib.ogv_render_blobs(None, 0, None, None, None, None, ctypes.byref(good), None, None, None) == 0
    for centres, radii, dens in [([], [], []), ([[0, 0, 0]], [0.0], [1.0]), ([[0, 0, 0]], [0.5], [-1.0]),
                                 ([[0, 0, 0]] * 17, [0.5] * 17, [1.0] * 17)]:
        f = api.blob_field(centres, radii, dens, [[1, 1, 1]] * len(centres))
        assert lib.ogv_render_blobs(None, 0, None, None, None, None, ctypes.byref(f), None, None, None) == -1
    assert lib.ogv_render_blobs(None, 0, None, None, None, None, None, None, None, None) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_refresh_rejects_null_arguments_on_host():
    from paper_2404_10272_amd import api
    assert api.lib().ogv_grid_refresh(None, None, None) == -1


def test_variant_names_map_to_header_values():
    # the binding's loop-variant names follow ogvdb.h's OGV_BRANCH, OGV_SKIP, OGV_VOXEL
    from paper_2404_10272_amd import api
    text = open(HEADER).read()
    vals = {k: int(v) for k, v in re.findall(r"#define (OGV_BRANCH|OGV_SKIP|OGV_VOXEL|OGV_SUBLEAF) (\d+)", text)}
    assert (api.BRANCH, api.SKIP, api.VOXEL, api.SUBLEAF) == (vals["OGV_BRANCH"], vals["OGV_SKIP"], vals["OGV_VOXEL"],
                                                              vals["OGV_SUBLEAF"])
    assert api._variant("voxel_branch") == api.BRANCH | api.VOXEL
    assert api._variant("voxel_skip") == api.SKIP | api.VOXEL
    assert api._variant("subleaf_skip") == api.SKIP | api.SUBLEAF
    assert api._variant(3) == 3
    for bad in (6, 8):
        with pytest.raises(ValueError):
            api._variant(bad)
    with pytest.raises(KeyError):
        api._variant("voxel")
