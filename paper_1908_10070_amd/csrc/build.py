"""Build libgbs.so (HIP kernels + host runtime, C ABI) for gfx950 with hipcc, in-tree.

Usage: python -m paper_1908_10070_amd.csrc.build [--force]
"""
import os
import pathlib
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = pathlib.Path(__file__).resolve().parent
PKG = HERE.parent
ROOT = PKG.parent
INCLUDE = ROOT / "include"
OUT = PKG / "libgbs.so"

# the engine kernels are split over several translation units so that they compile in parallel
SOURCES = ["gbs_eng_sqt.hip", "gbs_eng_sqt7.hip", "gbs_eng_grid5.hip", "gbs_eng_grid4.hip", "gbs_eng_quad.hip", "gbs_eng_tile.hip", "gbs_eng_strip.hip",
           "gbs_eng_dd.hip", "gbs_kernels.hip", "gbs_noalloc.hip", "gbs_sweep.hip", "gbs_runtime.cpp"]
HEADERS = ["gbs_internal.h", "gbs_tables.h", "gbs_engine_common.h", "gbs_quad_engine.h", "gbs_tile_engine.h",
           "gbs_qtile_engine.h", "gbs_strip_engine.h", "gbs_dd_engine.h", "gbs_sqt_engine.h", "gbs_chain_table.h"]

ARCH = "gfx950"
COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions stay off in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA results in VGPRs: the engines read every product back with VALU ops, so AGPR
    # destinations would cost one v_accvgpr_read per result register
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    f"-I{INCLUDE}", f"-I{HERE}",
]
# per-source flags: the double-double engine is built on error-free transformations (TwoSum, the
# fma product error), which a contracted a * b + c would silently break
EXTRA = {"gbs_eng_dd.hip": ["-ffp-contract=off"]}


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return p


def _stale() -> bool:
    if not OUT.exists():
        return True
    t = OUT.stat().st_mtime
    deps = [HERE / s for s in SOURCES + HEADERS] + [INCLUDE / "gbs.h"]
    return any(d.stat().st_mtime > t for d in deps)


def build(force: bool = True, verbose: bool = False, out: pathlib.Path = None, defines=()) -> pathlib.Path:
    """Compile every source and link libgbs.so (or `out`, with extra -D defines). Always recompiles
    when force is true."""
    out = pathlib.Path(out) if out else OUT
    if not force and out == OUT and not _stale():
        return OUT
    with tempfile.TemporaryDirectory(prefix="gbs_build_") as td:
        def compile_one(src):
            obj = pathlib.Path(td) / (src + ".o")
            lang = ["-x", "hip"] if src.endswith(".hip") else []
            cmd = [hipcc(), *COMMON, *EXTRA.get(src, []), *["-D" + d for d in defines], *lang, "-c", str(HERE / src),
                   "-o", str(obj)]
            if verbose:
                print(" ".join(cmd), flush=True)
            r = subprocess.run(cmd, capture_output=True, text=True)
            return src, obj, r

        jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
        with ThreadPoolExecutor(jobs) as pool:
            results = list(pool.map(compile_one, SOURCES))
        objs = []
        for src, obj, r in results:
            if r.returncode != 0:
                sys.stderr.write(r.stdout + r.stderr)
                raise RuntimeError(f"hipcc failed on {src}")
            objs.append(str(obj))
        tmp = out.with_name(out.name + f".tmp{os.getpid()}")
        cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", str(tmp), *objs]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("link of libgbs.so failed")
        os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(force=True, verbose="-v" in sys.argv))
