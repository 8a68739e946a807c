"""Build the gfx950 shared library libhgv.so from csrc/*.hip with hipcc.

Every .hip file is compiled to an object in parallel, then linked.  Run as
``python -m paper_1207_1773_amd.build`` or through ``__graft_entry__.build()``.
"""
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libhgv.so")
BUILD = os.path.join(ROOT, "_build", "hgv")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-result",
]


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src)[:-4] + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in l and "is not a recognized feature" not in l)
    return src, obj, r.returncode, msgs


def build(jobs=None, verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    jobs = jobs or min(len(srcs), os.cpu_count() or 4, 16)
    objs = []
    failed = False
    with cf.ThreadPoolExecutor(jobs) as ex:
        for src, obj, rc, msgs in ex.map(_compile, srcs):
            if msgs.strip() and (verbose or rc):
                print(msgs, file=sys.stderr)
            if rc:
                failed = True
                print("hipcc failed: %s" % src, file=sys.stderr)
            objs.append(obj)
    if failed:
        raise RuntimeError("HIP compilation failed")
    tmp = OUT + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
