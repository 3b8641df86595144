"""CPU checks of the C-ABI library: it loads, exports every function declared
in include/sm.h, its struct layouts match the header, and its defaults equal
the oracle's independently typed constants (no GPU calls here)."""
import ctypes
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "sm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sm_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    from paper_2606_14480_amd import sm
    lib = ctypes.CDLL(sm.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(sm.EXPORTS)


def test_struct_layouts():
    from paper_2606_14480_amd import sm
    assert sm.SEED_DTYPE.itemsize == 96
    assert sm.LONG_DTYPE.itemsize == 64
    assert ctypes.sizeof(sm.GhostNN) == 8 * (8 + 8 + 32 * 8 + 32 + 32 + 1)
    assert ctypes.sizeof(sm.Batch) == 8 + 16 + 11 * 8 + 8 + 3 * 8
    assert ctypes.sizeof(sm.Out) == 64


def test_defaults_agree_with_oracle(orc):
    from paper_2606_14480_amd import sm, events
    p, q = sm.default_params(), orc.default_params()
    for name, _ in sm.Params._fields_:
        if name.startswith("pad"):
            continue
        a, b = getattr(p, name), getattr(q, name)
        if name in sm.Params.ARRAYS:
            assert list(a) == list(b), name
        elif name == "ghost_nn":
            assert bytes(a) == bytes(b)
        else:
            assert a == b, name
    g, h = sm.default_geometry(), orc.default_geom()
    assert list(g.z) == list(h.z) == list(events.LAYER_Z)
    assert list(g.tan_stereo) == list(h.tan_a)
    assert list(g.ut_z) == list(h.ut_z) == list(events.UT_Z)
    assert list(g.ut_tan) == list(h.ut_tan)
    np.testing.assert_allclose(list(g.ut_tan), events.UT_TAN, rtol=1e-15)
    np.testing.assert_allclose(list(g.tan_stereo), events.LAYER_TAN, rtol=1e-15)
    assert g.z_ref == h.z_ref == events.Z_REF


def test_status_strings():
    from paper_2606_14480_amd import sm
    for s in range(0, -9, -1):
        assert sm.status_str(s) and sm.status_str(s) != "unknown status"
    assert sm.status_str(7) == "unknown status"


def test_product_does_not_touch_oracle():
    """The product package neither imports nor links the oracle."""
    pkg = os.path.join(ROOT, "paper_2606_14480_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                for bad in ("import oracle", "from oracle", "liboracle", "orc_"):
                    assert bad not in txt, (f, bad)


def test_create_rejects_bad_uv_settings():
    """Parameter checks come before any device call, so they run here."""
    from paper_2606_14480_amd import sm
    lib = sm.lib()
    for over in (dict(uv_mode=2), dict(uv_mode=1), dict(uv_mode=1, hough_bins=0), dict(uv_mode=1, hough_bins=129),
                 dict(uv_mode=1, hough_best=16, hough_fine=8), dict(uv_mode=1, hough_min=0),
                 dict(uv_mode=1, hough_fine=0)):
        p = sm.default_params(**over)
        h = ctypes.c_void_p()
        assert lib.sm_create(None, ctypes.byref(p), None, ctypes.byref(h)) == sm.ERR_INVALID, over
        assert not h.value


def test_create_rejects_bad_ut_settings():
    from paper_2606_14480_amd import sm
    lib = sm.lib()
    for over in (dict(ut_mode=2), dict(ut_mode=1, ut_min_hits=0), dict(ut_mode=1, ut_min_hits=5)):
        p = sm.default_params(**over)
        h = ctypes.c_void_p()
        assert lib.sm_create(None, ctypes.byref(p), None, ctypes.byref(h)) == sm.ERR_INVALID, over
        assert not h.value


def test_create_rejects_bad_final_selection():
    """final_sel outside {0, 1}, or the network form with an unusable network
    (a zero standardisation scale, a non-finite weight), is refused before any
    device call."""
    from paper_2606_14480_amd import sm
    lib = sm.lib()
    w = sm.ghost_nn_weights()
    zero_scale = dict(w, scale=[0.0] * 8)
    nan_w = dict(w, b2=float("nan"))
    for over in (dict(final_sel=2), dict(final_sel=-1), dict(final_sel=1, ghost_nn=zero_scale),
                 dict(final_sel=1, ghost_nn=nan_w), dict(final_sel=1, clone_gap=-0.1)):
        p = sm.default_params(**over)
        h = ctypes.c_void_p()
        assert lib.sm_create(None, ctypes.byref(p), None, ctypes.byref(h)) == sm.ERR_INVALID, over
        assert not h.value


def test_binding_structs_match_header(tmp_path):
    """Every ctypes mirror in the binding has the size and field offsets of
    its C struct in include/sm.h (compiled here with the host compiler)."""
    import os
    import subprocess

    from paper_2606_14480_amd import sm
    pairs = {"sm_geometry": sm.Geometry, "sm_params": sm.Params, "sm_config": sm.Config,
             "sm_batch": sm.Batch, "sm_kernel_times": sm.KernelTimes, "sm_out": sm.Out,
             "sm_ghost_nn": sm.GhostNN}
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "sm.h"', "int main(void) {"]
    for cname, py in pairs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    # the header is plain C: build it with gcc
    r = subprocess.run(["gcc", "-std=c11", "-I", inc, str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    got = {}
    for line in out.splitlines():
        cname, what, v = line.split()
        got[(cname, what)] = int(v)
    for cname, py in pairs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_context_refuses_single_workgroup():
    """A seeding grid below two workgroups is refused before any device call:
    the per-event form runs one workgroup per detector half on the
    per-workgroup scratch, which is sized by the grid."""
    import pytest
    from paper_2606_14480_amd import sm
    for w in (1, -3):
        with pytest.raises(sm.SmError) as e:
            sm.Context(seed_wgs=w)
        assert e.value.status == sm.ERR_INVALID
