"""Build librgf.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_1107_5300_amd.build   (or build() from Python)
"""

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librgf.so")

SOURCES = ["rgf_api.cpp", "rgf_lead.hip", "rgf_forward.hip", "rgf_adjoint.hip", "rgf_ldos.hip",
           "rgf_large.hip", "rgf_noalloc.hip", "rgf_segment.hip"]

HIP_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    # packed FP32 vector instructions stay off
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc():
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _stale(obj, src):
    """True if obj is missing or older than its source or any csrc header /
    include/rgf.h (every translation unit may include them)."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [os.path.join(CSRC, src), os.path.join(os.path.dirname(HERE), "include", "rgf.h")]
    deps += [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    return any(os.path.getmtime(d) > t for d in deps)


def _parse_remarks(text):
    """Per-kernel resource usage from -Rpass-analysis=kernel-resource-usage."""
    import re
    rec, cur = {}, None
    for line in text.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            rec[cur] = {}
            continue
        m = re.search(r"remark:\s+([^:]+): (\S+) \[", line)
        if m and cur:
            rec[cur][m.group(1).strip()] = m.group(2)
    return rec


def _demangle(names):
    try:
        r = subprocess.run(["c++filt"], input="\n".join(names).encode(), stdout=subprocess.PIPE,
                           stderr=subprocess.DEVNULL, timeout=60)
        out = r.stdout.decode().splitlines()
        if len(out) == len(names):
            return out
    except (OSError, subprocess.SubprocessError):
        pass
    return list(names)


def write_resource_report(objdir):
    """_build/kernel_resources.txt: VGPRs, scratch bytes per lane, spills and
    occupancy of every kernel, from the compiler's resource remarks."""
    rec = {}
    for src in SOURCES:
        path = os.path.join(objdir, os.path.splitext(src)[0] + ".remarks")
        if os.path.exists(path):
            with open(path) as fh:
                rec.update(_parse_remarks(fh.read()))
    names = sorted(rec)
    lines = ["kernel\tVGPRs\tAGPRs\tscratch_bytes_per_lane\tVGPR_spill\tSGPR_spill\twaves_per_SIMD"]
    for mangled, pretty in zip(names, _demangle(names)):
        r = rec[mangled]
        pretty = pretty.replace("rgf::(anonymous namespace)::", "").replace("(rgf::SweepArgs)", "")
        lines.append("\t".join([pretty, r.get("VGPRs", "?"), r.get("AGPRs", "?"),
                                r.get("ScratchSize [bytes/lane]", "?"), r.get("VGPRs Spill", "?"),
                                r.get("SGPRs Spill", "?"), r.get("Occupancy [waves/SIMD]", "?")]))
    with open(os.path.join(objdir, "kernel_resources.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


def build(verbose=False, jobs=None, incremental=False):
    """Compile every source to an object in parallel, then link librgf.so.
    incremental=True skips objects that are newer than their inputs (for
    development; the default always recompiles)."""
    cc = hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        if incremental and not _stale(obj, src):
            continue
        remarks = ["-Rpass-analysis=kernel-resource-usage"]
        cmd = [cc] + HIP_FLAGS + remarks + ["-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd = [cc, "-x", "hip"] + HIP_FLAGS + remarks + ["-c", os.path.join(CSRC, src),
                                                            "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, pr in procs:
        out, _ = pr.communicate()
        text = out.decode(errors="replace")
        with open(os.path.join(objdir, os.path.splitext(src)[0] + ".remarks"), "w") as fh:
            fh.write(text)
        lines = [ln for ln in text.splitlines()
                 if "packed-fp32-ops" not in ln and "kernel-resource-usage" not in ln]
        if pr.returncode != 0:
            failed.append((src, "\n".join(lines)))
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        msg = "\n".join(f"--- {s}\n{t}" for s, t in failed)
        raise RuntimeError("HIP build failed:\n" + msg)
    tmp = LIB + ".tmp"
    cmd = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-Wl,--no-undefined", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout.decode(errors="replace"))
    os.replace(tmp, LIB)
    write_resource_report(objdir)
    return LIB


def build_abi_check(verbose=False):
    """_build/abi_check: the host validation layer (rgf_api.cpp,
    rgf_noalloc.hip) rebuilt with AddressSanitizer and UndefinedBehavior-
    Sanitizer on the host side only, linked with the other objects of the
    normal build and driven by csrc/abi_check.cpp. Runs without a GPU.
    Returns the executable's path."""
    cc = hipcc()
    objdir = os.path.join(HERE, "_build")
    asan_dir = os.path.join(objdir, "asan")
    os.makedirs(asan_dir, exist_ok=True)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-g"]
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        if src in ("rgf_api.cpp", "rgf_noalloc.hip"):
            obj = os.path.join(asan_dir, os.path.splitext(src)[0] + ".o")
            cmd = [cc] + (["-x", "hip"] if src.endswith(".cpp") else []) + HIP_FLAGS + san + \
                  ["-c", os.path.join(CSRC, src), "-o", obj]
            r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
            if r.returncode != 0:
                raise RuntimeError("sanitizer build failed:\n" + r.stdout.decode(errors="replace"))
        elif not os.path.exists(obj):
            raise RuntimeError(f"{obj} missing: run build() first")
        objs.append(obj)
    exe = os.path.join(asan_dir, "abi_check")
    drv = os.path.join(asan_dir, "abi_check.o")
    r = subprocess.run([cc, "-x", "hip", "--offload-arch=gfx950", "-O1", "-std=c++17"] + san +
                       ["-c", os.path.join(CSRC, "abi_check.cpp"), "-o", drv],
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("sanitizer driver build failed:\n" + r.stdout.decode(errors="replace"))
    r = subprocess.run([cc, "--offload-arch=gfx950"] + san + ["-o", exe, drv] + objs,
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("sanitizer link failed:\n" + r.stdout.decode(errors="replace"))
    if verbose:
        print(exe)
    return exe


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv)
    print(LIB)
