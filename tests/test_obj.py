"""OBJ output of field lines (host code of the C-ABI library; runs without a GPU).

The file is the lines' exact text form: every vertex record reads back as the same FP32
value, and each line element lists its vertices' 1-based indices in order."""
import numpy as np
import pytest

import paper_2606_02627_amd as S


def parse_obj(path):
    verts, lines = [], []
    for row in open(path):
        parts = row.split()
        if not parts:
            continue
        if parts[0] == "v":
            verts.append([float(x) for x in parts[1:4]])
        elif parts[0] == "l":
            lines.append([int(x) for x in parts[1:]])
        else:
            raise AssertionError(f"unexpected record {row!r}")
    return np.array(verts, np.float64).reshape(-1, 3), lines


def test_obj_round_trips_every_vertex_and_line(tmp_path):
    rng = np.random.default_rng(2)
    lens = [3, 1, 0, 5, 2]
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    xyz = (rng.normal(size=(off[-1], 3)) * np.array([1e-7, 3.0, 7e5])).astype(np.float32)
    xyz[0] = [np.float32(1) / 3, -0.0, np.float32(2 ** -149)]  # many digits, signed zero, subnormal
    p = tmp_path / "lines.obj"
    n = S.streami_write_obj(str(p), off, xyz)
    assert n == off[-1]
    v, lines = parse_obj(p)
    np.testing.assert_array_equal(v.astype(np.float32), xyz)
    want = [list(range(off[i] + 1, off[i + 1] + 1)) for i in range(len(lens)) if lens[i] >= 2]
    assert lines == want


def test_obj_appends_into_one_joint_file(tmp_path):
    p = tmp_path / "joint.obj"
    a = np.arange(12, dtype=np.float32).reshape(4, 3)
    b = -np.arange(9, dtype=np.float32).reshape(3, 3)
    base = S.streami_write_obj(str(p), [0, 2, 4], a)
    base = S.streami_write_obj(str(p), [0, 3], b, append=True, vertex_base=base)
    assert base == 7
    v, lines = parse_obj(p)
    np.testing.assert_array_equal(v.astype(np.float32), np.concatenate([a, b]))
    assert lines == [[1, 2], [3, 4], [5, 6, 7]]
    # a new file (append = 0) starts over
    assert S.streami_write_obj(str(p), [0, 2], b[:2]) == 2
    assert parse_obj(p)[1] == [[1, 2]]


def test_obj_errors(tmp_path):
    with pytest.raises(S.StreamiError) as e:
        S.streami_write_obj(str(tmp_path / "no-such-dir" / "x.obj"), [0, 2], np.zeros((2, 3), np.float32))
    assert e.value.code == S.E_IO and "cannot open" in str(e.value)
    with pytest.raises(S.StreamiError) as e:
        S.streami_write_obj(str(tmp_path / "x.obj"), [0, 3, 2], np.zeros((3, 3), np.float32))
    assert e.value.code == S.E_ARG and "decrease" in str(e.value)
    with pytest.raises(S.StreamiError) as e:
        S.streami_write_obj_field(None, str(tmp_path / "x.obj"))
    assert e.value.code == S.E_ARG
