"""CPU checks of the C-ABI library: it loads, exports every declared symbol, and its host-only
functions and argument checks behave as documented. No kernel runs here."""
import os
import re

import numpy as np
import pytest

import paper_2105_08772_amd as lbm
from oracle import eos

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm_sc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_sc_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    L = lbm.load()
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(lbm.EXPORTS)


def test_critical_coupling_closed_forms():
    assert lbm.lbm_sc_gc(lbm.LBM_SC_PSI_EXP) == pytest.approx(-np.e ** 2, rel=1e-15)
    assert lbm.lbm_sc_gc(lbm.LBM_SC_PSI_ONEMINUS) == -4.0
    assert np.isnan(lbm.lbm_sc_gc(7))


@pytest.mark.parametrize("psi,ratio", [(0, 1.05), (0, 1.3), (0, 1.8), (1, 1.1), (1, 1.3)])
def test_coexistence_matches_oracle_rule(psi, ratio):
    ng, nl, p0 = lbm.lbm_sc_coexistence(psi, ratio)
    rg, rl, rp = eos.coexistence_rule(eos.G_of(ratio, psi), psi)
    assert abs(ng - rg) <= 1e-11 * rg
    assert abs(nl - rl) <= 1e-11 * rl
    assert abs(p0 - rp) <= 1e-11 * abs(rp)


def test_coexistence_rejects_supercritical():
    with pytest.raises(lbm.LbmScError) as e:
        lbm.lbm_sc_coexistence(0, 0.9)
    assert e.value.code == lbm.LBM_SC_EINVAL


BAD = [
    dict(nx=0), dict(tau=0.5), dict(psi=2), dict(geom=9), dict(prec=3), dict(radius=0.0),
    dict(width=0.0), dict(g_over_gc=0.95), dict(n_in=1.0, n_out=0.0), dict(noise_amp=-1.0),
    dict(geom=lbm.LBM_SC_SLAB, slab_thickness=0.0, slab_axis=2),
    dict(geom=lbm.LBM_SC_SLAB, slab_thickness=4.0, slab_axis=3), dict(packed_rows=2),
    dict(packed_rows=-1),
]


@pytest.mark.parametrize("bad", BAD)
def test_invalid_configurations_are_rejected_before_any_device_work(bad):
    kw = dict(radius=3.0, width=2.0)
    kw.update(bad)
    nx = kw.pop("nx", 8)
    cfg = lbm.config(nx, 8, 8, **kw)
    with pytest.raises(lbm.LbmScError) as e:
        lbm.lbm_sc_create(cfg)
    assert e.value.code == lbm.LBM_SC_EINVAL
    assert lbm.lbm_sc_last_error()


@pytest.mark.parametrize("dims,prec", [((1291, 1291, 1291), lbm.LBM_SC_FP32_SHIFTED),
                                       ((7600, 7600, 1), lbm.LBM_SC_FP32_SHIFTED),
                                       ((5400, 5400, 1), lbm.LBM_SC_FP64)])
def test_oversized_boxes_are_rejected_before_any_device_work(dims, prec):
    # more than 2^31 nodes; a z-plane whose 19 populations exceed 4 GiB (one buffer resource)
    cfg = lbm.config(*dims, prec=prec, radius=3.0, width=2.0)
    with pytest.raises(lbm.LbmScError) as e:
        lbm.lbm_sc_create(cfg)
    assert e.value.code == lbm.LBM_SC_EINVAL
    assert "2^31" in lbm.lbm_sc_last_error() or "4 GiB" in lbm.lbm_sc_last_error()


def test_population_bytes_is_one_buffer_of_the_device_bytes():
    for prec in (lbm.LBM_SC_FP64, lbm.LBM_SC_FP32_SHIFTED):
        cfg = lbm.config(40, 33, 12, prec=prec, radius=3.0, width=2.0)
        pb = lbm.lbm_sc_population_bytes(cfg)
        # two buffers, the last observed velocity (FP64, 24 B per node) and small arrays; the
        # device's shared observation workspace is not the box's
        n = 40 * 33 * 12
        extra = lbm.lbm_sc_device_bytes(cfg) - 2 * pb
        assert 24 * n < extra < 24 * n + (1 << 20)
        assert pb >= 19 * 40 * 33 * 12 * (8 if prec == lbm.LBM_SC_FP64 else 4)
        assert pb % 256 == 0
    with pytest.raises(lbm.LbmScError):
        lbm.lbm_sc_population_bytes(lbm.config(0, 4, 4))


def test_packed_rows_use_pitch_nx():
    """Packed rows store each z-plane's rows at pitch nx: the population buffer shrinks by the
    row padding (none when nx fills whole 128-byte lines)."""
    for prec, line in ((lbm.LBM_SC_FP32_SHIFTED, 32), (lbm.LBM_SC_FP64, 16)):
        for nx in (37, 64, 100, 129):
            pad = lbm.lbm_sc_population_bytes(lbm.config(nx, 20, 6, prec=prec, radius=3.0))
            pk = lbm.lbm_sc_population_bytes(lbm.config(nx, 20, 6, prec=prec, radius=3.0,
                                                        packed_rows=1))
            px = -(-nx // line) * line
            if nx % line == 0:
                assert pk == pad
            else:
                assert pk < pad
                # one z-plane's population planes: 19 x (pitch x ny rounded up to 64 elements)
                elem = 8 if prec == lbm.LBM_SC_FP64 else 4
                assert pk == 6 * 19 * (-(-(nx * 20) // 64) * 64) * elem
                assert pad == 6 * 19 * (-(-(px * 20) // 64) * 64) * elem


def test_sizes_of_the_largest_z_plane():
    # FP32, px = 7296: a 7296 x 7358 plane is the largest whose 19 populations (pitch rounded to
    # 64 elements plus a pad of a 19th of the plane rounded down to 256 B) stay under 4 GiB; the
    # byte counts exceed 2^32 and must come back whole, and one row more is invalid everywhere
    kw = dict(geom=lbm.LBM_SC_SLAB, prec=lbm.LBM_SC_FP32_SHIFTED, slab_thickness=3000.0,
              width=2.0)
    def pitch(ny):
        s = (7296 * ny + 63) // 64 * 64
        return s + s * 4 // 19 // 256 * 256 // 4
    pp = pitch(7358)
    assert 19 * pp * 4 < 2**32 <= 19 * pitch(7359) * 4
    cfg = lbm.config(7296, 7358, 2, **kw)
    assert lbm.lbm_sc_population_bytes(cfg) == 2 * 19 * pp * 4
    assert lbm.lbm_sc_device_bytes(cfg) > 2 * lbm.lbm_sc_population_bytes(cfg) > 2**33
    big = lbm.config(7296, 7359, 2, **kw)
    for f in (lbm.lbm_sc_population_bytes, lbm.lbm_sc_device_bytes, lbm.lbm_sc_create):
        with pytest.raises(lbm.LbmScError) as e:
            f(big)
        assert e.value.code == lbm.LBM_SC_EINVAL and "4 GiB" in lbm.lbm_sc_last_error()


def test_create_with_buffers_rejects_missing_buffers_before_any_device_work():
    cfg = lbm.config(8, 8, 8, radius=3.0, width=2.0)
    for a, b in ((0, 0), (0, 4096), (4096, 0)):
        with pytest.raises(lbm.LbmScError) as e:
            lbm.lbm_sc_create_with_buffers(cfg, a, b, 1 << 20)
        assert e.value.code == lbm.LBM_SC_EINVAL


def test_box_buffers_must_be_contiguous_device_tensors():
    import torch
    cfg = lbm.config(8, 8, 8, radius=3.0, width=2.0)
    host = torch.empty(1 << 20, dtype=torch.uint8)
    for bufs in ((host, host), (np.empty(16), np.empty(16))):
        with pytest.raises(ValueError):
            lbm.Box(cfg, buffers=bufs)


def test_ctypes_signatures_match_the_header():
    """Every prototype of include/lbm_sc.h against the argtypes and restype the Python binding
    gives the loaded library (a 64-bit return read as int truncates sizes of 2 GiB and more)."""
    import ctypes
    P = ctypes.POINTER
    structs = {"lbm_sc_config": lbm.LbmScConfig, "lbm_sc_obs": lbm.LbmScObs,
               "lbm_sc_info": lbm.LbmScInfo, "lbm_sc_launch": lbm.LbmScLaunch,
               "lbm_sc_group_launch": lbm.LbmScGroupLaunch}
    scalars = {"int": ctypes.c_int, "int32_t": ctypes.c_int32, "int64_t": ctypes.c_int64,
               "size_t": ctypes.c_size_t, "double": ctypes.c_double, "void": None}

    def ctype(decl, is_return):
        t = re.sub(r"\bconst\b", "", decl).strip()
        stars = t.count("*")
        base = t.replace("*", " ").split()[0]
        if stars == 0:
            return scalars[base]
        if stars == 1 and base == "char" and is_return:
            return ctypes.c_char_p
        if stars == 1 and base in structs:
            return P(structs[base])
        if stars == 1 and base in ("double", "int32_t", "int64_t"):
            return P(scalars[base])
        if stars == 1:           # opaque handles and raw device or host addresses
            return ctypes.c_void_p
        assert stars == 2, decl  # handle out-parameters and arrays of handles
        return P(ctypes.c_void_p)

    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"^#.*$", " ", text, flags=re.M)     # preprocessor lines
    protos = re.findall(r"([\w\s\*]+?)\b(lbm_sc_\w+)\s*\(([^)]*)\)\s*;", text)
    L = lbm.load()
    assert {name for _, name, _ in protos} == set(lbm.EXPORTS)
    for ret, name, args in protos:
        fn = getattr(L, name)
        assert fn.restype is ctype(ret, True), name
        # every parameter is named: drop the trailing name, keep the type
        want = [] if args.strip() in ("", "void") else [
            ctype(re.match(r"(.*?)\s*\b\w+$", a.strip()).group(1), False) for a in args.split(",")]
        assert list(fn.argtypes or []) == want, name


def test_ctypes_structs_match_the_c_layout(tmp_path):
    """Compile a probe against include/lbm_sc.h and compare every field offset and struct size
    with the ctypes mirrors of the Python binding."""
    import subprocess
    structs = {"lbm_sc_config": lbm.LbmScConfig, "lbm_sc_obs": lbm.LbmScObs,
               "lbm_sc_info": lbm.LbmScInfo, "lbm_sc_launch": lbm.LbmScLaunch,
               "lbm_sc_group_launch": lbm.LbmScGroupLaunch}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lbm_sc.h"', 'int main(void){']
    for cname, py in structs.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0;}")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    seen = 0
    for line in out:
        if not line:
            continue
        cname, fname, val = line.split()
        py = structs[cname]
        want = ctypes_sizeof(py) if fname == "sizeof" else getattr(py, fname).offset
        assert int(val) == want, (cname, fname)
        seen += 1
    assert seen == sum(len(p._fields_) + 1 for p in structs.values())


def ctypes_sizeof(t):
    import ctypes
    return ctypes.sizeof(t)


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_every_header_declaration_is_documented():
    """Each prototype of include/lbm_sc.h follows a comment block, directly or after the
    prototypes it shares that comment with (a set/get pair)."""
    lines = open(HEADER).read().splitlines()
    decl = re.compile(r"^(?:const\s+)?\w+\s*\*?\s*lbm_sc_\w+\s*\(")   # at column 0
    undocumented = []
    for k, line in enumerate(lines):
        if not decl.match(line):
            continue
        j = k - 1
        while j >= 0 and (decl.match(lines[j]) or lines[j].startswith((" ", "\t")) and
                          not lines[j].lstrip().startswith(("*", "/*"))):
            j -= 1            # earlier prototypes of the same group, or their continuation lines
        if j < 0 or not lines[j].rstrip().endswith("*/"):
            undocumented.append(line.strip())
    assert not undocumented, undocumented


def test_noalloc_step_checks_its_arguments_before_any_device_work():
    """The allocation-free multi-box step rejects more boxes than its fixed array holds, NULL
    boxes and unsupported launch shapes before touching a box or the device; no boxes is a
    no-op."""
    import ctypes
    base = dict(rows=2, z_chunk=32, xcd_remap=1, prefetch=0, persistent=0, workers=0,
                graph_steps=0, waves=4, tile_x=64, items_per_cu=0)
    lbm.lbm_sc_step_boxes_noalloc([], 4, **base)
    cases = [([ctypes.c_void_p(8)] * (lbm.LBM_SC_NOALLOC_MAX_BOXES + 1), base, "at most 1024"),
             ([ctypes.c_void_p(None)], base, "NULL"),
             ([], dict(base, rows=3), "unsupported launch shape"),
             ([], dict(base, persistent=1, workers=12), "workers")]
    for hs, launch, msg in cases:
        with pytest.raises(lbm.LbmScError) as e:
            lbm.lbm_sc_step_boxes_noalloc(hs, 2, **launch)
        assert e.value.code == lbm.LBM_SC_EINVAL
        assert msg in lbm.lbm_sc_last_error()
    with pytest.raises(lbm.LbmScError):
        lbm.lbm_sc_step_boxes_noalloc([], -1, **base)
