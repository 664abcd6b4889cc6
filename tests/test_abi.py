"""The C-ABI library loads on a host without a GPU, exports every function
that include/mpmq.h declares, and validates schemes / sizes on the host
(no compute call is made here)."""
import os
import re

import pytest

import workloads as WL

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mpmq.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mpmq_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import ctypes
    import paper_2207_04658_amd as mq
    lib = ctypes.CDLL(mq.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(mq.exported_symbols()) == names


def test_query_sizes_record_widths():
    import paper_2207_04658_amd as mq
    c1 = WL.c1()
    assert mq.mpmq_query_sizes(c1["scheme"], c1["params"], 8192)["words_per_particle"] == 7
    p3 = WL.c3_params()
    s3 = mq.mpmq_query_sizes(WL.scheme_c3(), p3, 300_000_000)
    assert s3["words_per_particle"] == 12 and s3["record_bits"] == 384
    assert s3["packed_bytes"] == 48 * 300_000_000
    f3 = mq.mpmq_query_sizes(WL.scheme_fp32(3), p3, 300_000_000)
    assert f3["packed_bytes"] == 96 * 300_000_000
    assert mq.mpmq_query_sizes(WL.scheme_c1(3, True), WL.c2()["params"], 1 << 20)["words_per_particle"] == 13
    # 512^3 grid of float4 nodes
    assert s3["grid_bytes"] == 32 * 512 ** 3  # 512^3 nodes of 4 int64 fixed-point sums
    assert s3["capacity_padded"] % 256 == 0


def test_query_sizes_agrees_with_oracle_layout(orc):
    import numpy as np
    import paper_2207_04658_amd as mq
    rng = np.random.default_rng(0)
    for dim in (2, 3):
        for _ in range(20):
            sc = WL.random_scheme(rng, dim)
            p = WL.params(dim, 64, 1e-4, 1e-6)
            q = mq.mpmq_query_sizes(sc, p, 1000)
            _, _, total, W = orc.layout(sc)
            assert (q["record_bits"], q["words_per_particle"]) == (total, W)


@pytest.mark.parametrize("mutate,msg", [
    (lambda s, p: s["fields"][0].update(bits=0), "bits"),
    (lambda s, p: s["fields"][1].update(hi=-30.0), "lo < hi"),
    (lambda s, p: s["fields"][2].update(rel_identity=True), "REL_IDENTITY"),
    (lambda s, p: s["fields"].__setitem__(3, WL.fixed("x", 8, 0, 1)), "exactly once"),
    (lambda s, p: s["fields"][1].update(kind="shared_exp", exp_bits=0), "exp_bits"),
    (lambda s, p: s["fields"][0].update(kind="raw_f32", bits=20), "RAW_F32"),
    (lambda s, p: p.update(grid_res=4), "grid_res"),
    (lambda s, p: p.update(dt=0.0), "dt"),
    (lambda s, p: p.update(dim=3), "dim"),
])
def test_invalid_arguments_rejected(mutate, msg):
    import paper_2207_04658_amd as mq
    c1 = WL.c1()
    s, p = c1["scheme"], dict(c1["params"])
    mutate(s, p)
    with pytest.raises(mq.MpmqError) as e:
        mq.mpmq_query_sizes(s, p, 100)
    assert e.value.status == -1 and msg in str(e.value)


def test_capacity_limits():
    import paper_2207_04658_amd as mq
    c1 = WL.c1()
    with pytest.raises(mq.MpmqError) as e:
        mq.mpmq_query_sizes(c1["scheme"], c1["params"], 0)
    assert e.value.status == -2
    with pytest.raises(mq.MpmqError):
        mq.mpmq_query_sizes(c1["scheme"], c1["params"], 1 << 32)


def test_record_too_long_rejected():
    import paper_2207_04658_amd as mq
    s = WL.scheme_fp32(3)
    s["fields"][0] = WL.fixed("x", 32, 0, 1)
    s["fields"][1] = WL.shared_exp("v", 32, 8, 20.0)  # 8 + 96 bits
    p = WL.params(3, 64, 1e-4, 1e-6)
    q = mq.mpmq_query_sizes(s, p, 10)
    assert q["record_bits"] == 96 + 104 + 288 + 288
