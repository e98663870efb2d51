"""CPU-side checks of the C-ABI library: it loads, exports every entry point
that include/*.h declares, and rejects invalid arguments before touching HIP."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[\w\s\*]+?\b(streami_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_five_entry_points():
    names = declared_functions()
    for n in ("streami_field_create", "streami_seed", "streami_advect", "streami_fetch_lines",
              "streami_fetch_outbox"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2606_02627_amd as S
    lib = S._load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_product_package_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_2606_02627_amd")
    for path in glob.glob(os.path.join(pkg, "**", "*"), recursive=True):
        if path.endswith((".py", ".hip", ".h", ".cpp")):
            src = open(path).read()
            assert "oracle" not in src.lower().replace("the oracle", ""), path


def _desc(**over):
    import fieldgen as fg
    import paper_2606_02627_amd as S
    b = fg.closed_form_block(lambda x, y, z: (0 * x + 1, 0 * x, 0 * x), (4, 4, 4))
    d = S.make_block_desc(b)
    for k, v in over.items():
        if isinstance(v, (list, tuple)):
            getattr(d, k)[:] = v
        else:
            setattr(d, k, v)
    return d


@pytest.mark.parametrize("field,value,msg", [
    ("dims", (0, 4, 4), "dims"), ("spacing", (1, -1, 1), "spacing"), ("ghost", 2, "ghost"),
    ("bounds_lo", (5, 0, 0), "bounds_lo"), ("rank_grid", (0, 1, 1), "rank_grid"),
    ("rank_coord", (1, 0, 0), "rank_coord"), ("boundary", 7, "boundary"),
    ("n_slices", 0, "n_slices"), ("nodes", None, "nodes"),
])
def test_field_create_rejects_invalid_descriptor(field, value, msg):
    import paper_2606_02627_amd as S
    d = _desc(**{field: value})
    with pytest.raises(S.StreamiError) as e:
        S.streami_field_create([d], S.F32)
    assert e.value.code == S.E_ARG and msg in str(e.value)


def test_field_create_rejects_bad_dtype_and_layout():
    import paper_2606_02627_amd as S
    with pytest.raises(S.StreamiError) as e:
        S.streami_field_create([_desc()], 9)
    assert e.value.code == S.E_ARG
    with pytest.raises(S.StreamiError) as e:
        S.streami_field_create([_desc()], S.F32, layout=99)
    assert e.value.code == S.E_ARG


def test_calls_on_null_handle_fail_cleanly():
    import paper_2606_02627_amd as S
    lib = S._load()
    null = ctypes.c_void_p(0)
    assert lib.streami_seed(null, 0, None, None, None, 1, None) == S.E_ARG
    assert lib.streami_advect(null, None, None) == S.E_ARG
    assert lib.streami_fetch_outbox(null, None, 0, None) == S.E_ARG
    assert lib.streami_fetch_lines(null, 0, 0, 0, None, None, 0, None, None, None, None) == S.E_ARG
    assert lib.streami_seed_batches(null, None, 1, None) == S.E_ARG
    assert lib.streami_forward(null, None, None) == S.E_ARG
    assert lib.streami_trace(null, None, 1, None, None) == S.E_ARG
    assert lib.streami_field_destroy(null) == S.OK
    assert b"NULL" in lib.streami_last_error()


def test_probe_rejects_invalid_arguments_before_device_work():
    """The memory probe validates everything before it touches HIP (the buffer pointer below
    is never dereferenced)."""
    import paper_2606_02627_amd as S
    lib = S._load()
    ms = ctypes.c_float()
    fake = ctypes.c_void_p(1 << 20)
    probe = lambda *a: lib.streami_probe_gather(*a, None, ctypes.byref(ms), None)
    assert probe(None, 1 << 20, 16, 64, 4, 16) == S.E_ARG
    assert probe(fake, 1 << 20, 24, 64, 4, 16) == S.E_ARG
    assert probe(fake, 1 << 20, 16, 64, 3, 16) == S.E_ARG
    assert probe(fake, 1 << 20, 16, 63, 4, 16) == S.E_ARG
    assert probe(fake, 1 << 20, 16, 64, 4, 0) == S.E_ARG
    assert probe(fake, 8, 16, 64, 4, 16) == S.E_ARG
    assert probe(fake, 1 << 40, 16, 64, 4, 16) == S.E_ARG
    assert b"record" in lib.streami_last_error()
    assert lib.streami_probe_valu(4, 32, None, ctypes.byref(ms), None) == S.E_ARG
    assert lib.streami_probe_valu(-1, 32, None, ctypes.byref(ms), None) == S.E_ARG
    assert lib.streami_probe_valu(0, 30, None, ctypes.byref(ms), None) == S.E_ARG
    assert lib.streami_probe_valu(0, 32, None, None, None) == S.E_ARG


STRUCTS = [("streami_block_desc", "BlockDesc"), ("streami_field_opts", "FieldOpts"),
           ("streami_seed_opts", "SeedOpts"), ("streami_seed_batch", "SeedBatch"), ("streami_shape", "Shape"), ("streami_hex_desc", "HexDesc"),
           ("streami_advect_params", "AdvectParams"),
           ("streami_stats", "Stats")]


def test_binding_structs_match_the_header_layout(tmp_path):
    """Every ctypes structure of the binding has the size and field offsets that a C
    compiler gives the header's struct (gcc on the header itself)."""
    import subprocess
    import paper_2606_02627_amd as S
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "streami.h"', "int main(void) {"]
    for cname, pyname in STRUCTS:
        lines.append(f'printf("{pyname} size %zu\\n", sizeof({cname}));')
        for fname, _ in getattr(S, pyname)._fields_:
            lines.append(f'printf("{pyname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for line in filter(None, out):
        pyname, what, val = line.split()
        cls = getattr(S, pyname)
        got = ctypes.sizeof(cls) if what == "size" else getattr(cls, what).offset
        assert got == int(val), (pyname, what, got, val)


@pytest.mark.parametrize("dims,dtype,layout,msg", [
    ((600, 600, 600), "f32", 0, "2 GiB"),   # 602^3 nodes x 12 B: one slice > 2 GiB
    ((1500, 1500, 2), "f32", 0, "16 MiB"),  # a z plane of 1502^2 x 12 B > 16 MiB
    ((1600, 1600, 2), "f16", 0, "16 MiB"),  # 1602^2 x 8 B (16-bit nodes padded to 8 B)
    ((300, 300, 300), "f32", 3, "2 GiB"),   # 301^3 cell records x 96 B > 2 GiB
    ((450, 450, 2), "f32", 3, "16 MiB"),    # a z plane of 451^2 cell records x 96 B > 16 MiB
    ((510, 510, 2), "f16", 5, "16 MiB"),    # a plane of 64^2 8^3-node bricks x 8 B = 2^24 B
])
def test_field_create_rejects_shapes_beyond_the_addressing_limits(dims, dtype, layout, msg):
    """The kernels address a slice with 32-bit byte offsets and 24-bit row/plane products;
    shapes beyond that are refused before any device work (the automatic layout falls
    back from cell records to node rows first)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("checked before device work; on a GPU machine a missed check would ingest")
    import paper_2606_02627_amd as S
    d = _desc(dims=dims)
    fmt = {"f32": S.F32, "f16": S.F16}[dtype]
    with pytest.raises(S.StreamiError) as e:
        S.streami_field_create([d], fmt, layout=layout)
    assert e.value.code == S.E_UNSUPPORTED and msg in str(e.value)


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_cell_layout_needs_fp32(dtype):
    """Cell records hold FP32 coefficients: a 16-bit field cannot use them."""
    import paper_2606_02627_amd as S
    with pytest.raises(S.StreamiError) as e:
        S.streami_field_create([_desc()], {"f16": S.F16, "bf16": S.BF16}[dtype], layout=S.LAYOUT_CELL)
    assert e.value.code == S.E_UNSUPPORTED and "FP32" in str(e.value)


def test_field_create_rejects_too_many_blocks():
    """The batched launch keeps the block table in at most 64 KiB of LDS: 315 blocks."""
    import paper_2606_02627_amd as S
    with pytest.raises(S.StreamiError) as e:
        S.streami_field_create([_desc()] * 316, S.F32)
    assert e.value.code == S.E_UNSUPPORTED and "315" in str(e.value)


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on exactly one GPU and says so for --gpus N > 1 (before any
    device work)."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2 and "one GPU" in r.stderr, (r.returncode, r.stderr[-500:])


def test_missing_library_fails_loudly():
    """Without the built HIP library every call raises ImportError naming the build step; there
    is no CPU fallback to run instead (checked in a child process so the loaded library of this
    one stays untouched)."""
    import subprocess
    import sys
    code = ("import paper_2606_02627_amd as s\n"
            "s.LIB_PATH = '/nonexistent/libstreami.so'\n"
            "s._lib = None\n"
            "try:\n"
            "    s._load()\n"
            "except ImportError as e:\n"
            "    print('ImportError:', e)\n"
            "else:\n"
            "    raise SystemExit('loaded')\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0 and "ImportError" in r.stdout and "build" in r.stdout, (r.stdout, r.stderr[-500:])


def test_hex_field_create_rejects_invalid_meshes():
    """Descriptor and mesh errors are found on the host, before any device work."""
    import fieldgen as fg
    import paper_2606_02627_amd as S
    good = fg.distorted_hex_mesh(18, (2, 2, 2), jitter=0.1)
    cases = [(dict(cells=np.where(good["cells"] == 5, 99, good["cells"]).astype(np.int32)), "names vertex"),
             (dict(lo=(1.0, 0.0, 0.0), hi=(0.5, 2.0, 2.0)), "lo < hi"),
             (dict(rank_coord=(0, 0, 3)), "rank_coord"),
             (dict(cells=good["cells"][:0]), "n_cells")]
    v = good["vertices"].copy()
    v[3, 1] = np.nan
    cases.append((dict(vertices=v), "not finite"))
    for change, msg in cases:
        with pytest.raises(S.StreamiError) as e:
            S.streami_field_create_hex(dict(good, **change))
        assert e.value.code == S.E_ARG and msg in str(e.value), (change, e.value)
