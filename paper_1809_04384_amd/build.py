"""Build the native library libdh2.so (HIP for gfx950 + host C++).

    python -m paper_1809_04384_amd.build

Objects go to paper_1809_04384_amd/_build/, the library to
paper_1809_04384_amd/libdh2.so.  Host structure code is compiled with
-ffp-contract=off (reproducible decisions); all HIP code with packed FP32
instructions disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdh2.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result", "-I" + os.path.join(ROCM, "include"),
          "-I" + os.path.join(HERE, "..", "include")]
HIPFLAGS = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-munsafe-fp-atomics"]
SOURCES = [
    ("plan.cpp", COMMON + ["-ffp-contract=off"], False),
    ("api.cpp", COMMON + ["-ffp-contract=off"], False),
    ("rank_model.cpp", COMMON, False),
    ("kernels.hip", COMMON + HIPFLAGS, True),
    ("matvec.hip", COMMON + HIPFLAGS, True),
    ("scratch.hip", COMMON + HIPFLAGS, True),
    ("rank_mlp.hip", COMMON + HIPFLAGS, True),
]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    lines = [l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l]
    if r.returncode != 0:
        sys.stderr.write("\n".join(lines) + "\n")
        raise RuntimeError("command failed: " + " ".join(cmd))
    return lines


def build(verbose=False):
    os.makedirs(OUT, exist_ok=True)
    objs = []
    for src, flags, is_hip in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(OUT, src + ".o")
        if is_hip:
            cmd = [HIPCC] + flags + ["-c", path, "-o", obj]
        else:
            # host-only translation units: HIP runtime headers, no device code
            cmd = [HIPCC] + flags + ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd))
        _run(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
