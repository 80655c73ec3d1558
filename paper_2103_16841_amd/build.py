"""Build the HIP library (libstb.so) in-tree for gfx950 with hipcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libstb.so")
SOURCES = [os.path.join(CSRC, "stb_lib.hip"), os.path.join(CSRC, "stb_pairs.hip"),
           os.path.join(CSRC, "stb_batch.hip"), os.path.join(CSRC, "stb_server.hip"),
           os.path.join(CSRC, "stb_apply.hip"),
           os.path.join(CSRC, "stb_faces.hip"), os.path.join(CSRC, "stb_solve.hip"),
           os.path.join(CSRC, "stb_dl.hip"), os.path.join(CSRC, "stb_proj.hip"),
           os.path.join(CSRC, "stb_scan.hip"), os.path.join(CSRC, "stb_tree.hip")]
HEADERS = [os.path.join(CSRC, "stb_device.h"), os.path.join(CSRC, "stb_internal.h"),
           os.path.join(CSRC, "stb_pairs.h"), os.path.join(ROOT, "include", "stb.h")]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]


def build(verbose=False):
    """Compile every HIP source into paper_2103_16841_amd/libstb.so."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc"] + FLAGS + ["-o", tmp] + SOURCES
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in res.stdout.splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + out)
    if verbose and out.strip():
        print(out)
    os.replace(tmp, LIB)
    return LIB


def stale():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose=True))
