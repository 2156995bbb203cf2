"""bench.py's command line on the host: more than one GPU is refused with a
message before anything touches a device."""
import pathlib
import subprocess
import sys

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", str(n)], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "measures one GPU" in r.stderr and f"--gpus {n}" in r.stderr
    assert r.stdout == ""


def test_bench_names_resolve():
    """Every global name a bench.py function reads exists at module level or in
    builtins (the GPU legs run only where a GPU is, so a missing helper would
    otherwise show there first)."""
    import builtins
    import symtable

    src = (ROOT / "bench.py").read_text()
    top = symtable.symtable(src, "bench.py", "exec")
    module_names = {s.get_name() for s in top.get_symbols() if s.is_assigned() or s.is_imported()}
    missing = []

    def walk(t):
        for s in t.get_symbols():
            if s.is_global() and s.is_referenced():
                n = s.get_name()
                if n not in module_names and not hasattr(builtins, n):
                    missing.append((t.get_name(), n))
        for c in t.get_children():
            walk(c)

    walk(top)
    assert not [m for m in missing if m[1] not in ("__file__",)], missing
