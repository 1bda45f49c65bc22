"""Build libnsasm.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2403_08777_amd.build [--resource-usage]

With --resource-usage the compiler's per-kernel resource remarks (VGPRs,
SGPRs, scratch bytes per lane, LDS bytes per workgroup, occupancy) are also
written to profiles/resources.json, tagged with a digest of the HIP sources so
that readers can tell whether it describes the current kernels.
"""

from __future__ import annotations

import hashlib
import json
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["runtime.hip", "sort.hip", "mesh.hip", "assemble.hip", "bandwidth.hip"]
LIB = os.path.join(HERE, "libnsasm.so")
ARCH = "gfx950"
RESOURCES = os.path.join(ROOT, "profiles", "resources.json")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
    "-munsafe-fp-atomics",
    # packed FP32 instructions stay disabled (known-bad on this platform)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def source_digest() -> str:
    """SHA-256 over the HIP sources (name and bytes, sorted by name)."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


_FIELDS = {"VGPRs": "vgprs", "AGPRs": "agprs", "TotalSGPRs": "sgprs", "ScratchSize [bytes/lane]": "scratch_bytes_per_lane",
           "Occupancy [waves/SIMD]": "occupancy_waves_per_simd", "LDS Size [bytes/block]": "lds_bytes_per_workgroup",
           "VGPRs Spill": "vgpr_spill", "SGPRs Spill": "sgpr_spill"}


def parse_resource_remarks(text: str) -> dict:
    """{kernel name (demangled, namespaces dropped): {field: int}} from the
    -Rpass-analysis=kernel-resource-usage remarks of one compilation."""
    out, cur = {}, None
    mangled = []
    for line in text.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            mangled.append(cur)
            out[cur] = {}
            continue
        m = re.search(r"remark:\s+([^:]+(?:\[[^\]]*\])?): (\S+) \[-Rpass", line)
        if m and cur and m.group(1).strip() in _FIELDS:
            v = m.group(2)
            out[cur][_FIELDS[m.group(1).strip()]] = int(v) if v.isdigit() else v
    if not mangled:
        return {}
    demangled = subprocess.run(["c++filt"], input="\n".join(mangled), capture_output=True, text=True,
                               check=True).stdout.splitlines()
    named = {}
    for mg, dm in zip(mangled, demangled):
        name = dm.replace("nsasm::(anonymous namespace)::", "")
        name = re.sub(r"^void ", "", name)
        name = re.match(r"([\w:]+(?:<[^()]*>)?)", name).group(1)
        named[name] = out[mg]
    return named


def build(resource_usage: bool = False, verbose: bool = False) -> str:
    """Compile every source to an object, link libnsasm.so; return its path."""
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    objs = []
    kernels = {}
    for src in SOURCES:
        obj = os.path.join(build_dir, src.replace(".hip", ".o"))
        cmd = [hipcc(), *HIPCC_FLAGS, f"-I{os.path.join(ROOT, 'include')}", "-c",
               os.path.join(CSRC, src), "-o", obj]
        if resource_usage:
            cmd.insert(1, "-Rpass-analysis=kernel-resource-usage")
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=resource_usage, text=True)
        if resource_usage:
            kernels.update(parse_resource_remarks(r.stderr))
            if r.returncode != 0:
                sys.stderr.write(r.stderr)
        if r.returncode != 0:
            raise subprocess.CalledProcessError(r.returncode, cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    if resource_usage:
        rec = {"source_sha256": source_digest(), "arch": ARCH,
               "command": "python -m paper_2403_08777_amd.build --resource-usage",
               "kernels": dict(sorted(kernels.items()))}
        with open(RESOURCES, "w") as f:
            json.dump(rec, f, indent=1)
            f.write("\n")
    return LIB


if __name__ == "__main__":
    path = build(resource_usage="--resource-usage" in sys.argv, verbose=True)
    print(path)
