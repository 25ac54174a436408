"""Host-side checks of the C ABI (no GPU): the library loads, exports every
entry point declared in include/gbp.h, and rejects bad input before any
device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def capi():
    from paper_2003_03134_amd import _capi
    return _capi


def test_header_declarations_are_exported(capi):
    text = open(os.path.join(ROOT, "include", "gbp.h")).read()
    declared = set(re.findall(r"\b(gbp_[a-z0-9_]+)\s*\(", text))
    lib = capi.load()
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert declared == set(capi.EXPORTS)


def test_header_constants_match_the_binding(capi):
    text = open(os.path.join(ROOT, "include", "gbp.h")).read()
    assert int(re.search(r"#define GBP_MLP_STATIC_MAX_BATCH (\d+)", text).group(1)) == \
        capi.GBP_MLP_STATIC_MAX_BATCH
    assert int(re.search(r"#define GBP_LOG_COLS (\d+)", text).group(1)) == capi.LOG_COLS
    assert int(re.search(r"#define GBP_MAX_BATCH_ITEMS (\d+)", text).group(1)) == capi.GBP_MAX_BATCH_ITEMS
    fields = re.search(r"typedef struct \{([^}]*)\} gbp_reproj;", text).group(1)
    names = re.findall(r"\b(?:double|int64_t)\s+(\w+);", fields)
    assert names == [n for n, _ in capi.gbp_reproj._fields_]


def test_default_options_are_the_papers(capi):
    lib = capi.load()
    o = capi.gbp_options()
    lib.gbp_default_options(C.byref(o))
    assert o.beta == 0.01 and o.relin_min_interval == 10 and o.undamped_after_relin == 8
    assert o.prior_anneal_iters == 10 and o.prior_weaken == 0.01
    assert o.precision == capi.GBP_FP32 and o.damp_mode == capi.GBP_DAMP_ETA


def _graph(capi, fkf, flm, nk=2, nl=2):
    fkf = np.ascontiguousarray(fkf, dtype=np.int32)
    flm = np.ascontiguousarray(flm, dtype=np.int32)
    kf = np.zeros((nk, 6))
    lm = np.ones((nl, 3))
    z = np.full((len(fkf), 2), 100.0)
    keep = [fkf, flm, kf, lm, z]
    g = capi.gbp_graph(nk, nl, len(fkf), fkf.ctypes.data_as(C.POINTER(C.c_int32)),
                       flm.ctypes.data_as(C.POINTER(C.c_int32)),
                       kf.ctypes.data_as(C.POINTER(C.c_double)),
                       lm.ctypes.data_as(C.POINTER(C.c_double)), None)
    m = capi.gbp_measurements(z.ctypes.data_as(C.POINTER(C.c_double)))
    return g, m, keep


@pytest.mark.parametrize("fkf,flm", [([0, 2], [0, 1]), ([0, 1], [0, 5]), ([-1, 0], [0, 0])])
def test_out_of_range_indices_are_rejected(capi, fkf, flm):
    lib = capi.load()
    g, m, keep = _graph(capi, fkf, flm)
    cam = capi.gbp_camera(500, 500, 320, 240, 1.0)
    h = C.c_void_p()
    st = lib.gbp_create(C.byref(g), C.byref(cam), C.byref(m), None, C.byref(h))
    assert st == capi.GBP_EINVAL
    assert b"out-of-range" in lib.gbp_last_error(h)
    # a failed problem refuses further work
    assert lib.gbp_iterate(h, 1, 0.4, 2.0) == capi.GBP_ESTATE
    lib.gbp_destroy(h)


def test_bad_options_are_rejected(capi):
    lib = capi.load()
    g, m, keep = _graph(capi, [0, 1], [0, 1])
    cam = capi.gbp_camera(500, 500, 320, 240, 1.0)
    o = capi.gbp_options()
    lib.gbp_default_options(C.byref(o))
    o.undamped_after_relin = 0
    h = C.c_void_p()
    assert lib.gbp_create(C.byref(g), C.byref(cam), C.byref(m), C.byref(o), C.byref(h)) == capi.GBP_EINVAL
    lib.gbp_destroy(h)
    o.undamped_after_relin = 8
    o.prior_anneal_iters = 65
    assert lib.gbp_create(C.byref(g), C.byref(cam), C.byref(m), C.byref(o), C.byref(h)) == capi.GBP_EINVAL
    lib.gbp_destroy(h)


def test_workspace_size_scales_with_factors(capi):
    lib = capi.load()
    g1, _, k1 = _graph(capi, [0, 1], [0, 1])
    n = C.c_size_t()
    assert lib.gbp_workspace_bytes(1, C.byref(g1), None, C.byref(n)) == 0
    small = n.value
    g2, _, k2 = _graph(capi, np.zeros(10000), np.zeros(10000))
    assert lib.gbp_workspace_bytes(1, C.byref(g2), None, C.byref(n)) == 0
    assert n.value > small + 10000 * 150


def test_packaged_damping_weights_load():
    """The shipped network file: BF16 copy is the rounding of the FP32
    master weights, every value finite, metadata present."""
    import numpy as np
    from paper_2003_03134_amd import learned
    bf16, theta, meta = learned.load_weights()
    u = theta.view(np.uint32).astype(np.uint64)
    expect = (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF).astype(np.uint16)
    assert np.array_equal(bf16, expect)
    assert np.all(np.isfinite(theta))
    assert meta["samples"] > 0 and meta["val_loss"][-1] < meta["val_loss"][0]


def test_static_training_step_rejects_oversized_batches(capi):
    """The allocation-free training step refuses a batch beyond its fixed
    scratch and bad arguments before touching a device (the pointers below
    are never dereferenced)."""
    lib = capi.load()
    fake = C.c_void_p(0x1000)
    n = capi.GBP_MLP_STATIC_MAX_BATCH + 1
    st = lib.gbp_mlp_train_step_static(fake, fake, fake, 10, fake, n, fake, fake, fake, fake,
                                       C.c_float(1e-3), 1, fake, fake, None)
    assert st == capi.GBP_EINVAL and b"exceeds" in lib.gbp_last_error(None)
    st = lib.gbp_mlp_train_step_static(fake, fake, fake, 10, fake, 0, fake, fake, fake, fake,
                                       C.c_float(1e-3), 1, fake, fake, None)
    assert st == capi.GBP_EINVAL


@pytest.mark.parametrize("entry", ["gbp_mlp_infer", "gbp_mlp_infer_bf16"])
def test_inference_rejects_misaligned_rows(capi, entry):
    """Feature rows are read as 16-byte vectors: a misaligned row pointer is
    refused before any device work (the pointers are never dereferenced);
    n = 0 with no buffers is a no-op."""
    lib = capi.load()
    fake = C.c_void_p(0x1000)
    st = getattr(lib, entry)(fake, C.c_void_p(0x1008), 4, fake, None, None)
    assert st == capi.GBP_EINVAL and b"aligned" in lib.gbp_last_error(None)
    st = getattr(lib, entry)(fake, fake, -1, fake, None, None)
    assert st == capi.GBP_EINVAL
    assert getattr(lib, entry)(None, None, 0, None, None, None) == capi.GBP_OK


def test_batches_beyond_the_index_limit_are_rejected(capi):
    """Totals over a batch (capacities included) above GBP_MAX_BATCH_ITEMS
    are refused before any array is read: the graphs below claim sizes their
    arrays do not have, and their pointers are never dereferenced."""
    lib = capi.load()
    lim = capi.GBP_MAX_BATCH_ITEMS
    fake_i = C.cast(C.c_void_p(0x1000), C.POINTER(C.c_int32))
    fake_d = C.cast(C.c_void_p(0x1000), C.POINTER(C.c_double))

    def graph(nk, nl, nf):
        return capi.gbp_graph(nk, nl, nf, fake_i, fake_i, fake_d, fake_d, None)

    n = C.c_size_t()
    # exactly at the limit: sized (about 400 GB in FP32), not refused
    g = graph(2, 2, lim)
    assert lib.gbp_workspace_bytes(1, C.byref(g), None, C.byref(n)) == 0
    assert n.value > 300 * lim
    # one factor more, split over two problems
    gs = (capi.gbp_graph * 2)(graph(2, 2, lim // 2), graph(2, 2, lim // 2 + 1))
    assert lib.gbp_workspace_bytes(2, gs, None, C.byref(n)) == capi.GBP_EINVAL
    assert b"batch too large" in lib.gbp_last_error(None)
    cams = (capi.gbp_camera * 2)(capi.gbp_camera(500, 500, 320, 240, 1.0), capi.gbp_camera(500, 500, 320, 240, 1.0))
    ms = (capi.gbp_measurements * 2)(capi.gbp_measurements(fake_d), capi.gbp_measurements(fake_d))
    h = C.c_void_p()
    assert lib.gbp_create_batch(2, gs, cams, ms, None, C.byref(h)) == capi.GBP_EINVAL
    assert b"batch too large" in lib.gbp_last_error(h)
    lib.gbp_destroy(h)
    # keyframes and landmarks, and a growth capacity beyond the limit
    for g in (graph(lim + 1, 2, 4), graph(2, lim + 1, 4)):
        assert lib.gbp_workspace_bytes(1, C.byref(g), None, C.byref(n)) == capi.GBP_EINVAL
    o = capi.gbp_options()
    lib.gbp_default_options(C.byref(o))
    o.max_factors = lim + 1
    g = graph(2, 2, 4)
    assert lib.gbp_workspace_bytes(1, C.byref(g), C.byref(o), C.byref(n)) == capi.GBP_EINVAL
    h = C.c_void_p()
    assert lib.gbp_create(C.byref(g), C.byref(cams[0]), C.byref(ms[0]), C.byref(o), C.byref(h)) == \
        capi.GBP_EINVAL
    assert b"batch too large" in lib.gbp_last_error(h)
    lib.gbp_destroy(h)
