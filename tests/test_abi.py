"""The C-ABI library loads and exports every entry point declared in
include/lbm.h; host-only paths (defaults, validation, sizes) behave as
documented.  No GPU compute is called here."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lbm():
    from paper_2101_11856_amd import lbm as L
    return L


def test_every_declared_symbol_is_exported(lbm):
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lbm.lib, n)]
    assert not missing, missing


def test_params_struct_matches_header(lbm):
    # field order and types of lbm_params as declared in the header
    text = open(HEADER).read()
    body = text[text.index("typedef struct {"):text.index("} lbm_params;")]
    fields = re.findall(r"^\s*(?:const\s+)?(\w+)\s*\*?\s*([a-z_0-9, \[\]]+);", body, flags=re.M)
    names = []
    for _t, decl in fields:
        for part in decl.split(","):
            names.append(re.sub(r"\[.*\]", "", part).strip())
    assert names == [f[0] for f in lbm.Params._fields_]
    assert C.sizeof(lbm.Params) == 8 * 20


def test_default_params_and_workspace_size(lbm):
    p = lbm.make_params(32, 32, 32, 0.01)
    assert p.s_bulk == 1.0 and list(p.s_high) == [1.0] * 4 and p.storage == lbm.F32
    n32 = lbm.workspace_size(p)
    # two population copies of 27 planes of 32^3 floats at least
    assert n32 >= 2 * 27 * 32 ** 3 * 4
    p16 = lbm.make_params(32, 32, 32, 0.01, storage="f16")
    p64 = lbm.make_params(32, 32, 32, 0.01, storage="f64")
    assert lbm.workspace_size(p16) < n32 < lbm.workspace_size(p64)


@pytest.mark.parametrize("kw,msg", [
    (dict(nx=0), "dimensions"),
    (dict(nu=0.0), "nu"),
    (dict(nu=float("nan")), "nu"),
    (dict(faces=(1, 0, 0, 0, 0, 0)), "both faces"),
    (dict(faces=(0, 0, 3, 3, 0, 0)), "INLET"),
    (dict(faces=(4, 4, 0, 0, 0, 0)), "OUTFLOW"),
    (dict(s_bulk=2.0), "s_bulk"),
    (dict(s_high=(1.0, 0.0, 1.0, 1.0)), "s_high"),
    (dict(storage=7), "storage"),
])
def test_invalid_params_rejected_before_any_launch(lbm, kw, msg):
    args = dict(nx=8, ny=8, nz=8, nu=0.1)
    args.update({k: v for k, v in kw.items() if k in args})
    extra = {k: v for k, v in kw.items() if k not in args}
    p = lbm.make_params(args["nx"], args["ny"], args["nz"], args["nu"], **extra)
    with pytest.raises(lbm.LbmError) as e:
        lbm.workspace_size(p)
    assert e.value.status == 1 and msg in str(e.value)


def test_non_periodic_axis_needs_two_nodes(lbm):
    p = lbm.make_params(1, 8, 8, 0.1, faces=(1, 1, 0, 0, 0, 0))
    with pytest.raises(lbm.LbmError):
        lbm.workspace_size(p)


def test_too_large_grid_rejected(lbm):
    p = lbm.make_params(2048, 2048, 1024, 0.1)
    with pytest.raises(lbm.LbmError) as e:
        lbm.workspace_size(p)
    assert "2^31" in str(e.value)


def test_create_rejects_small_or_misaligned_workspace(lbm):
    p = lbm.make_params(8, 8, 8, 0.1)
    h = C.c_void_p()
    st = lbm.lib.lbm_create(C.byref(p), C.c_void_p(256), 16, None, C.byref(h))
    assert st == 2 and not h.value
    st = lbm.lib.lbm_create(C.byref(p), C.c_void_p(260), 1 << 40, None, C.byref(h))
    assert st == 1 and b"aligned" in lbm.lib.lbm_last_error(None)


def test_version(lbm):
    assert "gfx950" in lbm.version()
