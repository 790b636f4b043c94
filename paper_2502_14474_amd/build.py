"""Build the C-ABI shared library libmdp.so for gfx950 with hipcc (in-tree).

Each source is compiled to an object of its own (in parallel, under _build/),
then the objects are linked into libmdp.so."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmdp.so")
OBJDIR = os.path.join(ROOT, "_build")
SOURCES = ["kernels.hip", "colblock.hip", "krylov.hip", "vecops.hip", "batch.hip", "api.cpp", "serve.cpp",
           "tune.cpp", "noalloc.hip", "devrows.hip", "arena.cpp", "xcdprod.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # one rounding per operation: every fused multiply-add is written out
    "-ffp-contract=off",
    # no packed float32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]
NOISE = ("unknown target feature", "packed-fp32-ops", "warning generated")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in (r.stdout + r.stderr).splitlines() if not any(n in ln for n in NOISE)]
    return r.returncode, msgs


def build(verbose=False, out=LIB, defines=()):
    os.makedirs(OBJDIR, exist_ok=True)
    tag = "" if not defines else "_" + str(abs(hash(tuple(defines))))
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC] + ["-D" + d for d in defines]
    jobs = []
    for s in SOURCES:
        obj = os.path.join(OBJDIR, os.path.splitext(s)[0] + tag + ".o")
        jobs.append((s, obj, [HIPCC] + FLAGS + inc + ["-c", os.path.join(CSRC, s), "-o", obj]))
    if verbose:
        for _, _, c in jobs:
            print(" ".join(c), flush=True)
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", "8"))))
    with ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(lambda j: (j[0],) + _run(j[2]), jobs))
    errors = [f"{s}:\n" + "\n".join(m) for s, rc, m in results if rc != 0]
    if errors:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errors))
    if verbose:
        for s, _, m in results:
            if m:
                print(f"{s}:\n" + "\n".join(m))
    tmp = out + ".tmp"
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [o for _, o, _ in jobs]
    if verbose:
        print(" ".join(link), flush=True)
    rc, msgs = _run(link)
    if rc != 0:
        raise RuntimeError("hipcc link failed:\n" + "\n".join(msgs))
    os.replace(tmp, out)
    return out


def build_probes(verbose=False):
    """Compile the stand-alone probes (paper_2502_14474_amd/probes/*.hip) to
    executables beside their sources: hardware ceilings the profiles quote."""
    outs = []
    d = os.path.join(HERE, "probes")
    for name in sorted(os.listdir(d)) if os.path.isdir(d) else []:
        if not name.endswith(".hip"):
            continue
        src = os.path.join(d, name)
        out = os.path.splitext(src)[0]
        cmd = [HIPCC] + [f for f in FLAGS if f != "-fPIC"] + [src, "-o", out]
        if verbose:
            print(" ".join(cmd), flush=True)
        rc, msgs = _run(cmd)
        if rc != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n" + "\n".join(msgs))
        outs.append(out)
    return outs


def build_code_objects(verbose=False, directory=os.path.join(ROOT, "tests", "kernels")):
    """Compile each .hip file of `directory` to a code object (.hsaco, gfx950)
    beside it: row kernels that tests hand to mdp_create_from_device_rows."""
    outs = []
    if not os.path.isdir(directory):
        return outs
    for name in sorted(os.listdir(directory)):
        if not name.endswith(".hip"):
            continue
        src = os.path.join(directory, name)
        out = os.path.splitext(src)[0] + ".hsaco"
        cmd = [HIPCC, "--genco"] + [f for f in FLAGS if f != "-fPIC"] + ["-I", os.path.join(ROOT, "include"),
                                                                        src, "-o", out]
        if verbose:
            print(" ".join(cmd), flush=True)
        rc, msgs = _run(cmd)
        if rc != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n" + "\n".join(msgs))
        outs.append(out)
    return outs


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
