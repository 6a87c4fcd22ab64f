"""CPU checks of the C ABI: the library loads and exports every declared entry
point; structure layouts agree with the header; defaults follow the paper."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "skmmse.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(skm_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    import paper_2205_11226_amd as skm
    names = declared_functions()
    assert len(names) >= 7
    so = ctypes.CDLL(skm.LIB_PATH)
    for n in names:
        assert hasattr(so, n), n


def test_struct_layouts():
    import paper_2205_11226_amd as skm
    from paper_2205_11226_amd.api import BlockInfo, Params
    assert ctypes.sizeof(Params) == 8 * 4 + 4 * 8 + 2 * 4
    assert ctypes.sizeof(BlockInfo) == skm.BLOCK_INFO_DTYPE.itemsize == 48


def test_defaults_follow_the_paper():
    import paper_2205_11226_amd as skm
    p = skm.default_params()
    assert (p.block, p.ring, p.window, p.expand_step) == (16, 4, 24, 4)
    assert p.sigma2 == 10.0 and (p.t_phi, p.t_nu) == (20.0, 0.1)
    q = skm.default_params(profile="excellent", mode="plain")
    assert (q.t_phi, q.t_nu, q.mode) == (20.0, 100.0, skm.MODES["plain"])


def test_create_reports_an_error_without_a_device():
    import torch
    import paper_2205_11226_amd as skm
    if torch.cuda.is_available():
        return
    try:
        skm.Context(0)
    except skm.SkmError as e:
        assert e.status in (-1, -3)
        assert skm.lib.skm_last_error()
    else:
        raise AssertionError("context creation without a GPU must fail")
