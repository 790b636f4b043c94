"""Installable package: the ctypes binding plus libmdp.so compiled for gfx950
and the C ABI header.  The build step runs paper_2502_14474_amd/build.py
(hipcc), so installing needs ROCm's hipcc but no GPU."""
import importlib.util
import os
import shutil

from setuptools import setup
from setuptools.command.build_py import build_py

ROOT = os.path.dirname(os.path.abspath(__file__))
PKG = "paper_2502_14474_amd"


class BuildPyWithHip(build_py):
    """Copy the Python sources, then compile the HIP library into the build
    tree's package and place the header beside it."""

    def run(self):
        super().run()
        spec = importlib.util.spec_from_file_location("mdp_build", os.path.join(ROOT, PKG, "build.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        dest = os.path.join(self.build_lib, PKG)
        os.makedirs(os.path.join(dest, "include"), exist_ok=True)
        mod.build(verbose=False, out=os.path.join(dest, "libmdp.so"))
        shutil.copy(os.path.join(ROOT, "include", "mdp.h"), os.path.join(dest, "include", "mdp.h"))


setup(
    name="mdp-mi355x",
    version="0.2.0",
    description="Inexact policy iteration for large discounted MDPs on MI355X (HIP, gfx950), C ABI + Python binding",
    packages=[PKG],
    python_requires=">=3.10",
    install_requires=["numpy"],
    cmdclass={"build_py": BuildPyWithHip},
    zip_safe=False,
)
