"""The oracle pins must catch plausible slips: each mutant of oracle.c (built
on the CPU into a temporary directory) has to make the pin suite fail, and so
does each mutant of the Python network and jump oracles (loaded in place of
the originals through tests/oracle_under_test.py)."""
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


MLP_SRC = os.path.join(ROOT, "oracle", "mlp.py")
SUR_SRC = os.path.join(ROOT, "oracle", "surrogate.py")
PY_MUTANTS = {
    # jump oracle
    "jump_big_step_uses_h": (SUR_SRC, "ref, st = field.step(x, jump * h, eps=eps)", "ref, st = field.step(x, h, eps=eps)"),
    "commutation_sign": (SUR_SRC, "lhs = xh + net(xh)", "lhs = xh - net(xh)"),
    "commutation_ref_from_x": (SUR_SRC, "ref, st = field.step(Y, h, eps=eps)", "ref, st = field.step(x, h, eps=eps)"),
    "accept_strict": (SUR_SRC, "accept = (r <= tol)", "accept = (r < tol)"),
    "activations_unrounded": (SUR_SRC, "round_act=omlp.round_bf16)", "round_act=None)"),
    "input_unrounded": (SUR_SRC, "xhat = omlp.round_bf16(omlp.normalise(x, self.period))",
                        "xhat = omlp.normalise(x, self.period)"),
    "fallback_one_step_short": (SUR_SRC, "tr = field.trace(x[rej], h, jump, eps=eps, keep_verts=False)",
                                "tr = field.trace(x[rej], h, jump - 1, eps=eps, keep_verts=False)"),
    "accepted_exit_ignored": (SUR_SRC, "code[accept & ~np.all((Y >= lo) & (Y < hi), axis=1)] = EXIT", "pass"),
    # network oracle
    "adam_m_bias_fixed_at_first_step": (MLP_SRC, "mhat = m[l][k] / (1 - b1 ** t)", "mhat = m[l][k] / (1 - b1)"),
    "adam_v_bias_off_by_one": (MLP_SRC, "vhat = v[l][k] / (1 - b2 ** t)", "vhat = v[l][k] / (1 - b2 ** (t + 1))"),
    "normalise_no_shift": (MLP_SRC, "return 2.0 * (np.mod(x, period) / period) - 1.0",
                           "return 2.0 * (np.mod(x, period) / period)"),
    "backward_dsilu_of_wrong_layer": (MLP_SRC, "dz = rg(dh * dsilu(zs[l - 1]))", "dz = rg(dh * dsilu(zs[l]))"),
    "rounding_skipped_for_activations": (MLP_SRC, "                h = round_act(h)\n", "                pass\n"),
}


@pytest.mark.parametrize("name", sorted(PY_MUTANTS))
def test_pins_catch_python_oracle_mutant(name, tmp_path):
    path, old, new = PY_MUTANTS[name]
    src = open(path).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    mpath = tmp_path / os.path.basename(path)
    mpath.write_text(src.replace(old, new))
    var = "STREAMI_MLP_ORACLE_SRC" if path == MLP_SRC else "STREAMI_SURROGATE_ORACLE_SRC"
    env = dict(os.environ, **{var: str(mpath)})
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_surrogate_oracle.py"),
                          os.path.join(ROOT, "tests", "test_mlp_oracle.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert res.returncode != 0, f"mutant {name} survived the pins:\n{res.stdout[-2000:]}"
