"""The oracle pins must catch plausible slips: each mutant of oracle.c (built
on the CPU into a temporary directory) has to make the pin suite fail."""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = {
    "rk4_weight_k2": ("(k1[c] + 2.0 * k2[c] + 2.0 * k3[c] + k4[c])", "(k1[c] + k2[c] + 2.0 * k3[c] + k4[c])"),
    "rk4_stage3_full_step": ("q[c] = p0[c] + 0.5 * h * k2[c];", "q[c] = p0[c] + h * k2[c];"),
    "rk4_sixth": ("(h / 6.0)", "(h / 5.0)"),
    "trilinear_axis_swap": ("double wt = w[0][a3] * w[1][b3] * w[2][c3];", "double wt = w[1][a3] * w[0][b3] * w[2][c3];"),
    "cell_index_round": ("int64_t k = (int64_t)floor(s);", "int64_t k = (int64_t)floor(s + 0.5);"),
    "node_stride_transposed": ("int64_t flat = slice_base + (iz[c3] * sy + iy[b3]) * sx + ix[a3];", "int64_t flat = slice_base + (ix[a3] * sy + iy[b3]) * sz + iz[c3];"),
    "max_steps_off_by_one": ("if (n >= m) {", "if (n > m) {"),
    "exit_closed_upper": ("if (!(x[a] >= b->lo[a] && x[a] < b->hi[a])) return 0;", "if (!(x[a] >= b->lo[a] && x[a] <= b->hi[a])) return 0;"),
    "dest_axis_mix": ("(r[0] + (int64_t)b->rank_grid[0] * (r[1] + (int64_t)b->rank_grid[1] * r[2]))", "(r[0] + (int64_t)b->rank_grid[1] * (r[1] + (int64_t)b->rank_grid[0] * r[2]))"),
    "time_blend_swapped": ("v[c] = (1.0 - al) * v0[c] + al * v1[c];", "v[c] = al * v0[c] + (1.0 - al) * v1[c];"),
    "time_blend_extrapolates": ("  if (al > 1) al = 1;\n", "\n"),
    "halo_miss_at_new_pos": ("io->out_dest[p] = orc_dest(b, fp);", "io->out_dest[p] = orc_dest(b, P);"),
    "stagnation_after_step": ("if (sqrt(k1[0] * k1[0] + k1[1] * k1[1] + k1[2] * k1[2]) < eps) return ORC_STAGNANT;", ""),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    mpath = tmp_path / "oracle_mut.c"
    mpath.write_text(src.replace(old, new))
    lib = str(tmp_path / "liboracle_mut.so")
    oracle.build(src=str(mpath), out=lib)
    env = dict(os.environ, STREAMI_ORACLE_LIB=lib)
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert res.returncode != 0, f"mutant {name} survived the pins:\n{res.stdout[-2000:]}"
