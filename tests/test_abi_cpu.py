"""Host-side checks of the C ABI: the library loads without a GPU and exports
every function that include/emg.h declares; the binding binds each one."""
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "emg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(emg_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_2001_04789_amd as emg
    declared = _declared()
    assert len(declared) >= 25
    out = subprocess.run(["nm", "-D", "--defined-only", emg.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\s[TW]\s+(emg_\w+)", out))
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    assert sorted(emg.SYMBOLS) == declared


def test_default_opts_without_gpu():
    import paper_2001_04789_amd as emg
    o = emg.default_opts()
    assert abs(o.rtol - 1e-10) < 1e-25 and o.nu1 == 2 and o.nu2 == 2 and abs(o.omega - 2 / 3) < 1e-15
    assert emg.lib.emg_last_error() is not None


def test_binding_fails_loudly_without_library(tmp_path):
    """The package refuses to import when libemg.so is absent (no CPU fallback)."""
    pkg = os.path.join(ROOT, "paper_2001_04789_amd")
    dst = tmp_path / "paper_2001_04789_amd"
    dst.mkdir()
    for f in ("__init__.py", "_abi.py"):
        (dst / f).write_text(open(os.path.join(pkg, f)).read())
    r = subprocess.run(["python", "-c", "import paper_2001_04789_amd"], cwd=tmp_path, capture_output=True, text=True)
    assert r.returncode != 0 and "not built" in r.stderr
