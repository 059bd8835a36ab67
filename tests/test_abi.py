"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
function include/idw.h declares, reports record sizes that match the layout arithmetic
printed in Sections 3.2-3.3, and rejects bad arguments before touching the device."""
import ctypes
import json
import os
import re

import pytest

from paper_1402_4986_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libidw.so not built")
    return _lib.load()


def test_every_declared_function_is_exported(lib):
    hdr = open(os.path.join(ROOT, "include", "idw.h")).read()
    declared = set(re.findall(r"\b(idw_[a-z_]+)\s*\(", hdr))
    assert declared == set(_lib.EXPORTED)
    for name in declared:
        assert hasattr(lib, name), name
    assert lib.idw_version().decode().startswith("idw-gfx950")


def test_batched_defaults_are_the_tuning_table(lib):
    # The build compiles the autotuner's chosen parameters in as the batched plans' defaults.
    tune = json.load(open(os.path.join(ROOT, "paper_1402_4986_amd", "tuning", "gfx950.json")))
    c, w = ctypes.c_int64(), ctypes.c_int32()
    assert lib.idw_batched_defaults(ctypes.byref(c), ctypes.byref(w)) == 0
    assert (c.value, w.value) == (tune["batch_chunk"], tune["batch_workgroups"])
    assert lib.idw_batched_defaults(None, ctypes.byref(w)) == _lib.IDW_EINVAL
    assert lib.idw_batched_plan_params(None, ctypes.byref(c), ctypes.byref(w)) == _lib.IDW_EINVAL


def _rb(lib, layout, dim, prec, is_data):
    b = (ctypes.c_size_t * 4)()
    rc = lib.idw_record_bytes(layout, dim, prec, is_data, b)
    return rc, list(b)


def test_record_sizes_follow_the_papers_layout_arithmetic(lib):
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_layout_arith.json")))
    # AoS: three 32-bit members, no padding (x, y, value for 2-D data).
    rc, b = _rb(lib, _lib.AOS, 2, _lib.FP32, 1)
    assert rc == 0 and b[0] * 8 == g["aos_record_members"] * g["member_bits_f32"]
    # AoaS FP32: aligned to 128 bits, hidden pad 128 - 3*32 = 32 bits.
    rc, b = _rb(lib, _lib.AOAS, 2, _lib.FP32, 1)
    assert rc == 0 and b[0] * 8 == g["aoas_alignment_bits"]
    assert b[0] * 8 - g["aos_record_members"] * g["member_bits_f32"] == g["aoas_f32_hidden_pad_bits"]
    # AoaS FP64: 64*3 + 64 = 2*128 bits.
    rc, b = _rb(lib, _lib.AOAS, 2, _lib.FP64, 1)
    assert rc == 0 and b[0] * 8 == g["aoas_f64_record_bits"]
    assert b[0] * 8 == 3 * 64 + g["aoas_f64_hidden_pad_bits"] == g["aoas_f64_accesses_of_128_bits"] * 128


def test_record_sizes_all_layouts(lib):
    assert _rb(lib, _lib.SOA, 3, _lib.FP32, 1) == (0, [4, 4, 4, 4])
    assert _rb(lib, _lib.SOA, 2, _lib.FP64, 0) == (0, [8, 8, 0, 0])
    assert _rb(lib, _lib.AOS, 3, _lib.FP32, 0) == (0, [12, 0, 0, 0])
    assert _rb(lib, _lib.AOAS, 3, _lib.FP32, 0) == (0, [16, 0, 0, 0])
    assert _rb(lib, _lib.HYBRID, 2, _lib.FP64, 1) == (0, [16, 8, 0, 0])
    assert _rb(lib, _lib.SOAOS, 2, _lib.FP64, 1) == (0, [16, 16, 0, 0])
    assert _rb(lib, _lib.SOAOS, 3, _lib.FP32, 1) == (0, [16, 8, 0, 0])
    assert _rb(lib, 9, 2, _lib.FP32, 1)[0] == _lib.IDW_EINVAL
    assert _rb(lib, _lib.SOA, 4, _lib.FP32, 1)[0] == _lib.IDW_EINVAL


def _pts(n, dim, layout, base=0x10000, stride=0x100000):
    s = _lib.IdwPoints()
    for k in range(4):
        s.ptr[k] = base + k * stride
    s.n, s.dim, s.layout = n, dim, layout
    return s


def _fwd(lib, data, query, p=2.0, prec=_lib.FP32, flags=0, ws=0x4000000, wsb=1 << 30, out=0x8000000):
    return lib.idw_forward(ctypes.byref(data), ctypes.byref(query), p, prec, flags, out, None, ws, wsb, None, None)


@pytest.mark.parametrize("case,code", [
    ("dim", _lib.IDW_EINVAL), ("p0", _lib.IDW_EINVAL), ("pnan", _lib.IDW_EINVAL), ("pbig", _lib.IDW_EINVAL),
    ("nulldata", _lib.IDW_EINVAL), ("n0", _lib.IDW_EINVAL), ("misaligned", _lib.IDW_EINVAL),
    ("layoutmix", _lib.IDW_EUNSUPPORTED), ("excl", _lib.IDW_EINVAL), ("prec", _lib.IDW_EINVAL),
    ("flags", _lib.IDW_EINVAL), ("ws", _lib.IDW_EWORKSPACE), ("wsalign", _lib.IDW_EWORKSPACE),
])
def test_bad_arguments_are_rejected_on_the_host(lib, case, code):
    d = _pts(1000, 2, _lib.AOAS)
    q = _pts(500, 2, _lib.AOAS, base=0x20000000)
    kw = {}
    if case == "dim":
        d.dim = q.dim = 4
    elif case == "p0":
        kw["p"] = 0.0
    elif case == "pnan":
        kw["p"] = float("nan")
    elif case == "pbig":
        kw["p"] = 65.0
    elif case == "nulldata":
        d.ptr[0] = None
    elif case == "n0":
        d.n = 0
    elif case == "misaligned":
        d.ptr[0] = 0x10008
    elif case == "layoutmix":
        q.layout = _lib.SOA
    elif case == "excl":
        kw["flags"] = _lib.EXCLUDE_SELF
    elif case == "prec":
        kw["prec"] = 7
    elif case == "flags":
        kw["flags"] = 0x40
    elif case == "ws":
        kw["wsb"] = 16
    elif case == "wsalign":
        kw["ws"] = 0x4000010
    rc = _fwd(lib, d, q, **kw)
    assert rc == code, lib.idw_last_error().decode()
    assert lib.idw_last_error().decode() != ""


def test_noalloc_forward_checks_its_scratch_limit_on_the_host(lib):
    # idw_forward_noalloc takes its workspace from a 64 MiB static device array: sizes whose
    # forward workspace exceeds it are refused before anything touches the device, as are
    # the arguments idw_forward refuses.
    def call(d, q, p=2.0, prec=_lib.FP32):
        return lib.idw_forward_noalloc(ctypes.byref(d), ctypes.byref(q), p, prec, 0, 0x8000000, None, None, None)
    b = ctypes.c_size_t()
    big_d, big_q = _pts(1 << 22, 2, _lib.AOAS), _pts(1 << 22, 2, _lib.AOAS, base=0x20000000)
    assert lib.idw_workspace_size(ctypes.byref(big_d), ctypes.byref(big_q), _lib.FP32, 0, None, ctypes.byref(b)) == 0
    assert b.value > 64 << 20
    assert call(big_d, big_q) == _lib.IDW_EWORKSPACE
    assert "scratch" in lib.idw_last_error().decode()
    d, q = _pts(1000, 2, _lib.AOAS), _pts(500, 2, _lib.AOAS, base=0x20000000)
    assert call(d, q, p=0.0) == _lib.IDW_EINVAL
    assert call(d, q, prec=7) == _lib.IDW_EINVAL
    q0 = _pts(0, 2, _lib.AOAS)
    assert call(d, q0) == 0                          # no queries: a no-op, as idw_forward
    # the benchmark size fits the scratch in both precisions once the data split is small
    # enough (the entry point takes the largest split that fits; the default one does not)
    for prec in (_lib.FP32, _lib.FP64):
        s = _pts(1 << 20, 2, _lib.AOAS)
        assert lib.idw_workspace_size(ctypes.byref(s), ctypes.byref(s), prec, 0, None, ctypes.byref(b)) == 0
        assert b.value > 64 << 20
        cfg = _lib.IdwConfig()
        cfg.split = 1
        assert lib.idw_workspace_size(ctypes.byref(s), ctypes.byref(s), prec, 0, ctypes.byref(cfg),
                                      ctypes.byref(b)) == 0
        assert b.value <= 64 << 20


def test_zero_queries_is_a_no_op(lib):
    d = _pts(1000, 3, _lib.SOA)
    q = _pts(0, 3, _lib.SOA)
    assert _fwd(lib, d, q, out=0) == 0


@pytest.mark.parametrize("n", [1, 1000, 1 << 16, 1 << 20, 1 << 24, 2 ** 31 - 1])
@pytest.mark.parametrize("m", [1, 1000, 1 << 16, 1 << 20, 1 << 24, 2 ** 31 - 1])
def test_adjoint_workspace_stays_bounded(lib, n, m):
    # The launch shapes grow the partial-sum arrays with the grid, each kept within 2 GiB
    # (or one row of the point set): the forward + adjoint workspace stays below
    # 4.5 GiB + 16 B per data point + 128 B per query at every size the boundary accepts.
    d, q = _pts(n, 2, _lib.AOAS), _pts(m, 2, _lib.AOAS, base=0x20000000)
    b = ctypes.c_size_t()
    flags = _lib.NEED_DZ | _lib.NEED_DP | _lib.NEED_DQ
    assert lib.idw_workspace_size(ctypes.byref(d), ctypes.byref(q), _lib.FP32, flags, None, ctypes.byref(b)) == 0
    assert b.value <= 4.5 * (1 << 30) + 16 * n + 128 * m


def test_workspace_size_grows_with_queries(lib):
    d = _pts(4096, 2, _lib.SOA)
    sizes = []
    for m in (1, 1000, 100000):
        q = _pts(m, 2, _lib.SOA)
        b = ctypes.c_size_t()
        assert lib.idw_workspace_size(ctypes.byref(d), ctypes.byref(q), _lib.FP32, 0, None, ctypes.byref(b)) == 0
        f = ctypes.c_size_t()
        assert lib.idw_workspace_size(ctypes.byref(d), ctypes.byref(q), _lib.FP32, _lib.NEED_DZ, None,
                                      ctypes.byref(f)) == 0
        assert f.value > b.value  # the adjoint needs more than the forward
        x = ctypes.c_size_t()
        assert lib.idw_workspace_size(ctypes.byref(d), ctypes.byref(q), _lib.FP32, _lib.NEED_DX, None,
                                      ctypes.byref(x)) == 0
        assert x.value > f.value  # the data-coordinate partials come after the rest
        sizes.append(b.value)
    assert sizes[0] < sizes[1] < sizes[2]


def test_backward_argument_checks(lib):
    d = _pts(1000, 2, _lib.HYBRID)
    q = _pts(10, 2, _lib.HYBRID, base=0x20000000)
    args = [ctypes.byref(d), ctypes.byref(q), 2.0, _lib.FP32]
    rc = lib.idw_backward(*args, 0, 1, 1, 1, None, None, None, None, 0x4000000, 1 << 30, None, None)
    assert rc == _lib.IDW_EINVAL  # no gradient requested
    rc = lib.idw_backward(*args, _lib.NEED_DZ, 1, 1, 1, None, None, None, None, 0x4000000, 1 << 30, None, None)
    assert rc == _lib.IDW_EINVAL  # grad_z missing
    rc = lib.idw_backward(*args, _lib.NEED_DX, 1, 1, 1, None, None, None, None, 0x4000000, 1 << 30, None, None)
    assert rc == _lib.IDW_EINVAL  # grad_x missing
    rc = lib.idw_backward(*args, 0x20, 1, 1, 1, None, None, None, None, 0x4000000, 1 << 30, None, None)
    assert rc == _lib.IDW_EINVAL  # unknown flag bit


def test_batched_is_declared(lib):
    plan = ctypes.c_void_p()
    rc = lib.idw_batched_plan_create(None, 0, _lib.FP32, None, ctypes.byref(plan))
    assert rc != 0


def test_timing_interface_without_device(lib):
    ms, cnt = ctypes.c_double(-1.0), ctypes.c_int64(-1)
    assert lib.idw_timing_enable(1) == 0
    assert lib.idw_timing_read(_lib.T_FWD_SWEEP, ctypes.byref(ms), ctypes.byref(cnt)) == 0
    assert ms.value == 0.0 and cnt.value == 0
    assert lib.idw_timing_read(9, ctypes.byref(ms), ctypes.byref(cnt)) == _lib.IDW_EINVAL
    assert lib.idw_timing_enable(0) == 0


def test_batched_plan_argument_checks(lib):
    plan = ctypes.c_void_p()
    arr = (_lib.IdwInstance * 2)()
    for k in range(2):
        arr[k].data = _pts(1000, 2, _lib.AOAS)
        arr[k].query = _pts(100, 2, _lib.AOAS, base=0x20000000)
        arr[k].p = 2.0
        arr[k].out_z = 0x30000000
    # FP64 plans are not offered
    assert lib.idw_batched_plan_create(arr, 2, _lib.FP64, None, ctypes.byref(plan)) == _lib.IDW_EUNSUPPORTED
    # only aligned-AoS records
    arr[1].data.layout = _lib.SOA
    arr[1].query.layout = _lib.SOA
    rc = lib.idw_batched_plan_create(arr, 2, _lib.FP32, None, ctypes.byref(plan))
    assert rc == _lib.IDW_EUNSUPPORTED and b"instance 1" in lib.idw_last_error()
    arr[1].data.layout = _lib.AOAS
    arr[1].query.layout = _lib.AOAS
    arr[0].p = -1.0
    rc = lib.idw_batched_plan_create(arr, 2, _lib.FP32, None, ctypes.byref(plan))
    assert rc == _lib.IDW_EINVAL and b"instance 0" in lib.idw_last_error()
    assert not plan.value


def test_kahan_precision_is_fp32_storage_with_its_own_limits(lib):
    # IDW_FP32_KAHAN stores FP32 records, builds only 4 queries per lane, and batched
    # plans do not take it.
    for layout in (_lib.SOA, _lib.AOS, _lib.AOAS, _lib.HYBRID, _lib.SOAOS):
        assert _rb(lib, layout, 3, _lib.FP32_KAHAN, 1) == _rb(lib, layout, 3, _lib.FP32, 1)
    d = _pts(1000, 2, _lib.AOAS)
    q = _pts(500, 2, _lib.AOAS, base=0x20000000)
    cfg = _lib.IdwConfig()
    cfg.queries_per_lane = 8
    rc = lib.idw_forward(ctypes.byref(d), ctypes.byref(q), 2.0, _lib.FP32_KAHAN, 0, 0x8000000, None, 0x4000000,
                         1 << 30, None, ctypes.byref(cfg))
    assert rc == _lib.IDW_EUNSUPPORTED
    plan = ctypes.c_void_p()
    arr = (_lib.IdwInstance * 1)()
    arr[0].data = d
    arr[0].query = q
    arr[0].p = 2.0
    arr[0].out_z = 0x30000000
    assert lib.idw_batched_plan_create(arr, 1, _lib.FP32_KAHAN, None, ctypes.byref(plan)) == _lib.IDW_EUNSUPPORTED


def test_queries_per_lane_builds(lib):
    # FP32 builds 2, 4 and 8 queries per lane, but the relative-weight sweep (p >= 6) only 4
    # and 8; FP64 builds 2 and 4.  Refused combinations fail on the host with
    # IDW_EUNSUPPORTED before anything is enqueued (null stream, fake device pointers).
    d = _pts(1000, 2, _lib.AOAS)
    q = _pts(500, 2, _lib.AOAS, base=0x20000000)
    cfg = _lib.IdwConfig()
    for prec, qpl, p in ((_lib.FP32, 2, 8.0), (_lib.FP32, 16, 2.0), (_lib.FP64, 8, 2.0), (_lib.FP32_KAHAN, 2, 2.0)):
        cfg.queries_per_lane = qpl
        rc = lib.idw_forward(ctypes.byref(d), ctypes.byref(q), p, prec, 0, 0x8000000, None, 0x4000000, 1 << 30,
                             None, ctypes.byref(cfg))
        assert rc == _lib.IDW_EUNSUPPORTED, (prec, qpl, p)
        assert "queries_per_lane" in lib.idw_last_error().decode()


@pytest.mark.parametrize("field,value", [("reserved", 1), ("split", -1), ("queries_per_lane", -4),
                                         ("batch_chunk", -1), ("separate_adjoint", 2), ("near_search", 2),
                                         ("near_search", -1)])
def test_config_fields_are_validated(lib, field, value):
    d = _pts(1000, 2, _lib.AOAS)
    q = _pts(500, 2, _lib.AOAS, base=0x20000000)
    cfg = _lib.IdwConfig()
    if field == "reserved":
        cfg.reserved[1] = value
    else:
        setattr(cfg, field, value)
    b = ctypes.c_size_t()
    assert lib.idw_workspace_size(ctypes.byref(d), ctypes.byref(q), _lib.FP32, 0, ctypes.byref(cfg),
                                  ctypes.byref(b)) == _lib.IDW_EINVAL
    rc = lib.idw_forward(ctypes.byref(d), ctypes.byref(q), 2.0, _lib.FP32, 0, 0x8000000, None, 0x4000000,
                         1 << 30, None, ctypes.byref(cfg))
    assert rc == _lib.IDW_EINVAL
    rc = lib.idw_backward(ctypes.byref(d), ctypes.byref(q), 2.0, _lib.FP32, _lib.NEED_DZ, 1, 1, 1, 0x9000000,
                          None, None, None, 0x4000000, 1 << 30, None, ctypes.byref(cfg))
    assert rc == _lib.IDW_EINVAL
