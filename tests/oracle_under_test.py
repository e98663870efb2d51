"""The Python oracle modules a pin test runs against: the package's own, or -- when
the mutant test points an environment variable at a modified copy -- that copy,
so that the pins can be shown to catch plausible slips in the Python oracles."""
import importlib.util
import os

from oracle import mlp as _mlp
from oracle import surrogate as _surrogate


def _exec(path, name):
    spec = importlib.util.spec_from_file_location(f"oracle.{name}", path)
    mod = importlib.util.module_from_spec(spec)  # package "oracle": relative imports resolve
    spec.loader.exec_module(mod)
    return mod


_mlp_src = os.environ.get("STREAMI_MLP_ORACLE_SRC")
_sur_src = os.environ.get("STREAMI_SURROGATE_ORACLE_SRC")
mlp = _exec(_mlp_src, "mlp_under_test") if _mlp_src else _mlp
if _sur_src or _mlp_src:
    surrogate = _exec(_sur_src or _surrogate.__file__, "surrogate_under_test")
    surrogate.omlp = mlp  # the jump oracle evaluates the network under test
else:
    surrogate = _surrogate
