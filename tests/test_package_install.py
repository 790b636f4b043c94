"""The package installs offline from a checkout (pyproject.toml + setup.py,
whose build step compiles the HIP library with hipcc; no GPU needed) and the
installed module exports every function the installed header declares."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions(path):
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mdp_[a-z_0-9]+)\s*\(", text)) - {"mdp_rows_fn"})


def test_pip_install_offline_exports_the_header(tmp_path):
    target = tmp_path / "site"
    r = subprocess.run([sys.executable, "-m", "pip", "install", "--no-build-isolation", "--no-deps",
                        "--no-index", "--target", str(target), ROOT],
                       capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    pkg = target / "paper_2502_14474_amd"
    assert (pkg / "libmdp.so").is_file() and (pkg / "include" / "mdp.h").is_file()
    code = ("import json, paper_2502_14474_amd as m\n"
            "from paper_2502_14474_amd import native\n"
            "lib = native.load()\n"
            "print(json.dumps({'file': m.__file__, 'lib': native.LIB_PATH, 'names': sorted(native.SIGNATURES),"
            " 'missing': [n for n in native.SIGNATURES if not hasattr(lib, n)],"
            " 'version': lib.mdp_version().decode()}))\n")
    env = dict(os.environ, PYTHONPATH=str(target))
    r = subprocess.run([sys.executable, "-c", code], cwd=str(tmp_path), env=env, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    import json
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["file"].startswith(str(pkg)) and out["lib"].startswith(str(pkg))
    assert out["missing"] == []
    assert out["names"] == _header_functions(pkg / "include" / "mdp.h")
    assert "gfx950" in out["version"]
