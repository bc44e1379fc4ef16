"""Build libabilu.so (HIP, gfx950) in-tree: paper_1912_00539_amd/lib/libabilu.so."""
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUTDIR = os.path.join(HERE, "lib")
OUT = os.path.join(OUTDIR, "libabilu.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"


def torch_lib_dir():
    """Directory of the HIP runtime that torch loads (torch ships its own libamdhip64.so).

    The library must use the same HIP runtime instance as the process's torch: device
    pointers and streams created by one HIP runtime are unknown to another."""
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.submodule_search_locations:
        return None
    d = os.path.join(list(spec.submodule_search_locations)[0], "lib")
    return d if os.path.exists(os.path.join(d, "libamdhip64.so")) else None


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = True, jobs: int = 8) -> str:
    os.makedirs(OUTDIR, exist_ok=True)
    objdir = os.path.join(OUTDIR, "obj")
    os.makedirs(objdir, exist_ok=True)
    common = [HIPCC, f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-I", INCLUDE, "-I", CSRC,
              "-mcode-object-version=5",
              # packed FP32 instructions stay off (v_pk_* f32 forms)
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Wall", "-Wno-unused-function"]
    procs, objs = [], []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = common + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd)))
        if len(procs) >= jobs:
            src0, p0 = procs.pop(0)
            if p0.wait() != 0:
                raise RuntimeError(f"hipcc failed on {src0}")
    for src0, p0 in procs:
        if p0.wait() != 0:
            raise RuntimeError(f"hipcc failed on {src0}")
    # host-only C++ (orderings)
    for src in sorted(glob.glob(os.path.join(CSRC, "*.cpp"))):
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-I", INCLUDE, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
    tl = torch_lib_dir()
    if tl:
        # link against torch's HIP runtime: NEEDED libamdhip64.so resolves to the copy torch loaded
        link = ["g++", "-shared", "-fPIC", "-o", OUT + ".tmp"] + objs + [
            f"-L{tl}", "-l:libamdhip64.so", f"-Wl,-rpath,{tl}", "-Wl,--no-undefined"]
    else:
        link = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", OUT + ".tmp"] + objs
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(OUT + ".tmp", OUT)
    build_c_solve(tl, verbose)
    return OUT


C_SOLVE = os.path.join(OUTDIR, "abilu_c_solve")


def build_c_solve(tl, verbose: bool = True) -> str:
    """The C-only user of the ABI (tests/c_abi/solve.c): plain C, linked against libabilu.so
    (found next to it) and the same HIP runtime."""
    src = os.path.join(ROOT, "tests", "c_abi", "solve.c")
    if not os.path.exists(src):
        return ""
    rocm_inc = os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(HIPCC))), "include")
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__", "-I", rocm_inc, "-I", INCLUDE,
           src, "-o", C_SOLVE + ".tmp", f"-L{OUTDIR}", "-labilu", "-Wl,-rpath,$ORIGIN", "-lm"]
    if tl:
        cmd[-1:-1] = [f"-L{tl}", "-l:libamdhip64.so", f"-Wl,-rpath,{tl}"]
    else:
        cmd[-1:-1] = ["-L/opt/rocm/lib", "-lamdhip64"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(C_SOLVE + ".tmp", C_SOLVE)
    return C_SOLVE


if __name__ == "__main__":
    build()
    sys.exit(0)
