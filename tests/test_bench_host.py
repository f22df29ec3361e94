"""Host checks of bench.py (no GPU): the module imports, and every bare name
it calls resolves to one of its own functions, an import, a builtin or a
name bound in the calling scope, so a leg that no GPU test runs still has
the functions it calls."""
import ast
import builtins
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _load():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _bound_names(fn):
    """Arguments and names assigned, imported or defined anywhere in fn."""
    out = set()
    for node in ast.walk(fn):
        if isinstance(node, ast.arg):
            out.add(node.arg)
        elif isinstance(node, ast.Name) and isinstance(node.ctx, ast.Store):
            out.add(node.id)
        elif isinstance(node, (ast.FunctionDef, ast.Lambda)) and hasattr(node, "name"):
            out.add(node.name)
        elif isinstance(node, (ast.Import, ast.ImportFrom)):
            for a in node.names:
                out.add((a.asname or a.name).split(".")[0])
    return out


def test_bench_imports_and_every_called_name_resolves():
    mod = _load()
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    missing = []
    for fn in [n for n in tree.body if isinstance(n, ast.FunctionDef)]:
        local = _bound_names(fn)
        for node in ast.walk(fn):
            if isinstance(node, ast.Call) and isinstance(node.func, ast.Name):
                name = node.func.id
                if name in local or hasattr(mod, name) or hasattr(builtins, name):
                    continue
                missing.append(f"{fn.name}: {name}")
    assert not missing, missing


def test_bench_legs_defined():
    mod = _load()
    for leg in ("run_batched", "run_precision", "run_dense", "run_field", "run_scenes", "run_neural",
                "run_served", "main"):
        assert callable(getattr(mod, leg, None)), leg
