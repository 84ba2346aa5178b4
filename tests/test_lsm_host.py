"""CPU tests of liblsm.so: exported symbols and the host-side logic (lattice
builder, spring typing, argument validation).  No GPU calls are made."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

from oracle import Net, Params
from paper_2201_04565_amd import inputs, lsm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NAN = float("nan")


def header_functions():
    names = set()
    for hdr in os.listdir(os.path.join(ROOT, "include")):
        if hdr.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", hdr)).read()
            names |= set(re.findall(r"^(?:int|void|const char \*)\s*(lsm_\w+)\(", txt, re.M))
    return sorted(names)


def test_library_exports_every_header_function():
    L = lsm.load_library()
    names = header_functions()
    assert len(names) >= 20
    for nm in names:
        assert hasattr(L, nm), nm
    from paper_2201_04565_amd import cnn
    assert set(names) == set(lsm.EXPORTS) | set(lsm.BATCH_EXPORTS) | set(cnn.CNN_EXPORTS)


def _model(img, wl, **over):
    kw = dict(k=wl["k"], s=wl["s"], mass=wl["mass"], a=wl.get("a", 1.0),
              k_face=wl.get("k_face", 1.0), k_diag=wl.get("k_diag", 1.0),
              void_value=wl.get("void_value", -1), precision=wl.get("precision", "fp64"))
    kw.update(over)
    return lsm.HostModel(img, **kw)


def _oracle(img, wl, **over):
    kw = dict(k=wl["k"], s=wl["s"], mass=wl["mass"], a=wl.get("a", 1.0),
              k_face=wl.get("k_face", 1.0), k_diag=wl.get("k_diag", 1.0),
              void_value=wl.get("void_value", -1))
    kw.update(over)
    return Net.lattice(img, Params(**kw))


CASES = [
    ("c1", lambda: inputs.c1_image()),
    ("c2", lambda: inputs.brick_and_mortar(150, 97, seed=1)),
    ("c4", lambda: inputs.circular_inclusions(64, seed=1003)),
    ("c3", lambda: inputs.gaussian_random_field_3d(24, corr_len=3.0, seed=2)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_builder_matches_oracle(name, make):
    img = make()
    wl = inputs.WORKLOADS[name]
    g = _model(img, wl)
    o = _oracle(img, wl)
    assert (g.n, g.m) == (o.n, o.m)
    gs, os_ = g.springs(), o.springs()
    assert np.array_equal(gs["p"], os_["p"]) and np.array_equal(gs["q"], os_["q"])
    assert np.allclose(gs["k"], os_["k"], rtol=1e-15, atol=0)
    assert np.allclose(gs["r0"], os_["r0"], rtol=1e-14, atol=0)
    assert np.allclose(gs["rc"], os_["rc"], rtol=1e-14, atol=0)
    assert np.allclose(g.X0, o.X0, rtol=0, atol=1e-12)


def test_c2_full_size_counts():
    # closed form (W-1) H + (2W-1)(H-1) at 2048^2
    g = _model(inputs.c2_image(), inputs.WORKLOADS["c2"])
    assert (g.n, g.m) == (4194304, 12574721)
    # algorithmic bytes per launch of the default two-step sweep (two steps):
    # 24 B state read + written, flag, break byte read + written per site
    assert g.step_bytes() == 4194304 * 51
    # the single-step sweep rewrites a break byte only when it changes
    g.set_launch("sweep")
    assert g.step_bytes() == 4194304 * 50


def test_3d_step_bytes_count_the_particle_list():
    # 3D fp32k: u (24 B) and v (12 B) read and written, flag, 4-byte break
    # mask, and the packed coordinates of the one-thread-per-particle launch
    # -- or the eight 16-bit row entries of the LDS-window kernel
    img = inputs.gaussian_random_field_3d(24, seed=3)
    wl = inputs.WORKLOADS["c3"]
    g = _model(img, wl, precision="fp32k")
    assert g.n == int((img != inputs.VOID).sum()) > 0
    assert g.launch_variant() == "compact"
    assert g.step_bytes() == g.n * (2 * (24 + 12) + 1 + 4 + 16)
    g.set_launch("compact_direct")
    assert g.step_bytes() == g.n * (2 * (24 + 12) + 1 + 4 + 4)
    g64 = _model(img, wl, precision="fp64")
    assert g64.step_bytes() == g64.n * (2 * (24 + 24) + 1 + 4 + 16)
    g64.set_launch("gather")
    assert g64.step_bytes() == g64.n * (2 * (24 + 24) + 1 + 4 + 4)


def test_small_kernel_variant_rules():
    # the one-workgroup kernel: 2D lattices whose state fits its LDS
    wl = inputs.WORKLOADS["c1"]
    _model(inputs.c1_image(), wl).set_launch("small")
    _model(inputs.c1_image(), wl, precision="fp32k").set_launch("small")
    with pytest.raises(lsm.LsmError):
        _model(inputs.bernoulli_two_phase(64, 64, 0.3, seed=1), wl).set_launch("small")
    img3 = inputs.gaussian_random_field_3d(12, seed=3)
    with pytest.raises(lsm.LsmError):
        _model(img3, inputs.WORKLOADS["c3"]).set_launch("small")


def test_compact_kernel_variant_rules():
    # the compact per-particle layout of the 3D interior steps: 3D only
    img3 = inputs.gaussian_random_field_3d(12, seed=3)
    _model(img3, inputs.WORKLOADS["c3"]).set_launch("compact")
    _model(img3, inputs.WORKLOADS["c3"], precision="fp32k").set_launch("compact")
    with pytest.raises(lsm.LsmError):
        _model(inputs.c1_image(), inputs.WORKLOADS["c1"]).set_launch("compact")
    with pytest.raises(lsm.LsmError):
        _model(inputs.c1_image(), inputs.WORKLOADS["c1"]).set_launch("compact_direct")


def test_compact_kernel_stages_windows_where_they_fit():
    # single-phase lattices stage their neighbours in LDS windows; two
    # phases, or a window of 2^15 particles or more, read them directly
    wl3 = inputs.WORKLOADS["c3"]
    g = _model(inputs.gaussian_random_field_3d(20, seed=2), wl3)
    assert g.launch_variant() == "compact"
    g.set_launch("compact_direct")
    assert g.launch_variant() == "compact_direct"
    g.set_launch("compact")
    assert g.launch_variant() == "compact"
    rng = np.random.default_rng(1)
    two = dict(wl3, k=[[1.0, float("nan")], [float("nan"), 0.3]], s=[[0.03, float("nan")], [float("nan"), 0.08]],
               mass=[1.0, 2.0])
    assert _model(rng.integers(0, 2, size=(6, 7, 8)).astype(np.uint8), two).launch_variant() == "compact_direct"
    # a sparse plane (one particle every 128 sites) under a full one: the
    # first workgroup's 256 particles span 32,768 sites of plane 0, so its
    # window in plane 1 holds more than 2^15 particles
    img = np.zeros((2, 40, 1024), np.uint8)
    img[0].reshape(-1)[np.arange(0, 40 * 1024) % 128 != 0] = inputs.VOID
    assert _model(img, wl3).launch_variant() == "compact_direct"
    img[0] = inputs.VOID
    img[0, :, :64] = 0
    assert _model(img, wl3).launch_variant() == "compact"


def test_table2_paper_mode_types():
    # explicit interface constants (paper's spring table), r0 = 10
    k = [[2e-5, 1.25e-4], [1.25e-4, 2e-3]]
    s = [[0.1, 0.04], [0.04, 0.01]]
    img = np.array([[1, 0, 1], [0, 1, 0]], np.uint8)
    g = lsm.HostModel(img, k=k, s=s, mass=[1.0, 1.0], a=10.0)
    sp = g.springs()
    ph = img.ravel()
    for p, q, kk, rc in zip(sp["p"], sp["q"], sp["k"], sp["rc"]):
        a, b = sorted((ph[p], ph[q]))
        assert kk == k[a][b]
        assert rc == pytest.approx(10.0 * (1 + s[a][b]), rel=1e-15)


@pytest.mark.parametrize("bad", [
    dict(mass=[0.0, 1.0]), dict(dt=0.0), dict(gamma=-1.0), dict(a=-1.0),
    dict(k=[[-1.0, NAN], [NAN, 1.0]]), dict(s=[[NAN, NAN], [NAN, 0.1]]),
])
def test_create_rejects_bad_config(bad):
    kw = dict(k=[[0.1, NAN], [NAN, 1.0]], s=[[0.2, NAN], [NAN, 0.05]], mass=[1.0, 1.0])
    kw.update(bad)
    with pytest.raises(lsm.LsmError) as e:
        lsm.HostModel(np.zeros((4, 4), np.uint8), **kw)
    assert e.value.code == lsm.LSM_EINVAL


def test_build_rejects_bad_image():
    kw = dict(k=[[1.0]], s=[[0.1]], mass=[1.0])
    with pytest.raises(lsm.LsmError) as e:
        lsm.HostModel(np.full((3, 3), 7, np.uint8), **kw)   # phase 7 with one phase
    assert e.value.code == lsm.LSM_EINVAL


def test_empty_and_degenerate_images():
    kw = dict(k=[[1.0]], s=[[0.1]], mass=[1.0], void_value=255)
    g = lsm.HostModel(np.full((3, 5), 255, np.uint8), **kw)
    assert (g.n, g.m) == (0, 0)
    g = lsm.HostModel(np.zeros((1, 1), np.uint8), **kw)
    assert (g.n, g.m) == (1, 0)
    g = lsm.HostModel(np.zeros((1, 7), np.uint8), **kw)
    assert (g.n, g.m) == (7, 6)


def test_batch_rejects_more_sites_than_the_sweep_addresses():
    # the row sweeps use 32-bit byte offsets into 16-byte site records: a
    # batch holds fewer than 2^28 sites (sizes are checked before any image
    # is read, so tiny buffers stand in for the images here)
    L = lsm._load_batch(lsm.load_library())
    cfg = lsm.make_config(lattice=lsm.TRI2D, k=[[1.0]], s=[[0.1]], mass=[1.0])
    img = np.zeros(16, np.uint8)
    ptrs = (C.c_void_p * 2)(img.ctypes.data, img.ctypes.data)
    h = C.c_void_p()
    dims = np.array([[16384, 8192, 1], [16384, 8192, 1]], dtype=np.int64)
    assert L.lsm_batch_create(C.byref(cfg), 2, ptrs, dims.ctypes.data_as(C.c_void_p),
                              C.byref(h)) == lsm.LSM_EINVAL


def test_unbound_calls_report_state_errors():
    L = lsm.load_library()
    g = lsm.HostModel(np.zeros((4, 4), np.uint8), k=[[1.0]], s=[[0.1]], mass=[1.0])
    assert L.lsm_apply_strain_increment(g._h, 0.01) == lsm.LSM_ESTATE
    assert L.lsm_relax(g._h, 10) == lsm.LSM_ESTATE
    R = lsm.Record()
    assert L.lsm_read_state(g._h, C.byref(R)) == lsm.LSM_ESTATE
    assert L.lsm_bind(g._h, None, 0, None) == lsm.LSM_EINVAL
    assert L.lsm_strerror(lsm.LSM_EUNSTABLE).decode().startswith("non-finite")


def test_cnn_layout_matches_oracle_definition():
    from oracle import cnn_oracle as co
    from paper_2201_04565_amd import cnn
    L = cnn._load()
    cfg = cnn.CnnConfig(8, 32, 32, (C.c_int32 * 5)(32, 64, 128, 128, 256), 256, 65)
    h = C.c_void_p()
    assert L.lsm_cnn_create(C.byref(cfg), C.byref(h)) == 0
    n = C.c_int64()
    L.lsm_cnn_param_count(h, C.byref(n))
    spec, n_or = co.layout([32, 64, 128, 128, 256], 256, 65)
    assert n.value == n_or
    wo = np.zeros(7, np.int64); bo = np.zeros(7, np.int64); wn = np.zeros(7, np.int64)
    L.lsm_cnn_layout(h, wo.ctypes.data_as(C.c_void_p), bo.ctypes.data_as(C.c_void_p),
                     wn.ctypes.data_as(C.c_void_p))
    for l, sp in enumerate(spec):
        assert (wo[l], wn[l]) == sp["w"] and bo[l] == sp["b"][0]
    bad = cnn.CnnConfig(8, 24, 24, (C.c_int32 * 5)(32, 64, 128, 128, 256), 256, 65)
    h2 = C.c_void_p()
    assert L.lsm_cnn_create(C.byref(bad), C.byref(h2)) == lsm.LSM_EINVAL
    L.lsm_cnn_destroy(h)
