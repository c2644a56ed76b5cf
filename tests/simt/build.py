"""Host build of the library with its kernels run on the CPU (test
infrastructure only; the product library is the gfx950 build of
paper_1711_08013_amd/build.py).

The library source is compiled as plain C++ against the stand-in runtime in
tests/simt/include/hip/hip_runtime.h, for an emulated device of
SIMT_CU_COUNT (default 256) compute units whose occupancy and static LDS per
kernel are those the gfx950 build of the same source reports.  Two
mechanical edits are made to a copy of it: each triple-chevron launch becomes a call of simt::launch with
the kernel call in a lambda, and every array of the device arena gets an
allocation of its own.  The build uses the host address sanitizer, so every
device-memory access of the kernels is bounds-checked against the
allocation it belongs to."""
from __future__ import annotations

import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1711_08013_amd", "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libosqp_simt.so")
CLANG = os.environ.get("SIMT_CXX", "/opt/rocm/llvm/bin/clang++")
SEPARATE_ARRAYS = os.environ.get("SIMT_ONE_ARENA", "") == ""
# the server launches from its scheduler thread, one launch at a time, which
# the stand-in runtime (one scheduler, launches run when issued) allows
WITH_SERVER = os.environ.get("SIMT_NO_SERVER", "") == ""


def asan_runtime() -> str:
    """Path of the sanitizer runtime to preload into a Python process that
    loads the library."""
    out = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"],
                         capture_output=True, text=True, check=True).stdout.strip()
    if not os.path.isabs(out) or not os.path.exists(out):
        raise RuntimeError("address-sanitizer runtime not found next to " + CLANG)
    return out


def _split_top(s: str) -> list[str]:
    parts, depth, cur = [], 0, []
    for ch in s:
        if ch in "([{":
            depth += 1
        elif ch in ")]}":
            depth -= 1
        if ch == "," and depth == 0:
            parts.append("".join(cur).strip())
            cur = []
        else:
            cur.append(ch)
    parts.append("".join(cur).strip())
    return parts


_LAUNCH = re.compile(r"([A-Za-z_]\w*(?:<[^<>;()]*>)?)<<<(.*?)>>>\((.*?)\);", re.S)


def translate(src: str) -> str:
    def repl(m: re.Match) -> str:
        cfg = _split_top(m.group(2))
        grid, block = cfg[0], cfg[1]
        return (f"::simt::launch(dim3({grid}), dim3({block}), [&]() {{ "
                f"{m.group(1)}({m.group(3)}); }});")

    out, n = _LAUNCH.subn(repl, src)
    if n == 0 or "<<<" in out:
        raise RuntimeError("launch translation failed")
    if not WITH_SERVER:
        out = out.replace('#include "server.h"', "// server left out of the host build")
    # every array of the device arena gets an allocation of its own (rounded
    # up to the 16-byte load width), so the sanitizer bounds each array, not
    # only the arena
    arena = "T *p = reinterpret_cast<T *>(base + used);"
    if SEPARATE_ARRAYS:
        if arena not in out:
            raise RuntimeError("arena allocation not found")
        out = out.replace(arena, "T *p = base ? static_cast<T *>(::simt_array_alloc(count * sizeof(T)))"
                                 " : reinterpret_cast<T *>(base + used);")
    return out + GRAPH_BINDERS


# binders of the kernels the library puts into graphs or launches
# cooperatively (argument types as in their definitions)
GRAPH_BINDERS = r"""
namespace {
template <class T>
bool simt_bind_kernels() {
  using namespace osqpmi;
  ::simt::register_kernel((const void *)solve_wg_kernel<T>, [](void **a) {
    Batch<T> b = *static_cast<Batch<T> *>(a[0]);
    const int *list = *static_cast<const int **>(a[1]);
    const int nl = *static_cast<int *>(a[2]), slot = *static_cast<int *>(a[3]);
    return std::function<void()>([=]() { solve_wg_kernel<T>(b, list, nl, slot); });
  });
  ::simt::register_kernel((const void *)polish_wg_kernel<T>, [](void **a) {
    Batch<T> b = *static_cast<Batch<T> *>(a[0]);
    const int *list = *static_cast<const int **>(a[1]);
    const int nl = *static_cast<int *>(a[2]), slot = *static_cast<int *>(a[3]);
    double *ws = *static_cast<double **>(a[4]);
    const long long stride = *static_cast<long long *>(a[5]);
    const int rmax = *static_cast<int *>(a[6]);
    return std::function<void()>([=]() { polish_wg_kernel<T>(b, list, nl, slot, ws, stride, rmax); });
  });
  ::simt::register_kernel((const void *)solve_grid_kernel<T>, [](void **a) {
    Batch<T> b = *static_cast<Batch<T> *>(a[0]);
    const int *list = *static_cast<const int **>(a[1]);
    const int nl = *static_cast<int *>(a[2]);
    double *partials = *static_cast<double **>(a[3]);
    GridBarrier *bar = *static_cast<GridBarrier **>(a[4]);
    return std::function<void()>([=]() { solve_grid_kernel<T>(b, list, nl, partials, bar); });
  });
  ::simt::register_kernel((const void *)scale_grid_kernel<T>, [](void **a) {
    Batch<T> b = *static_cast<Batch<T> *>(a[0]);
    const int *list = *static_cast<const int **>(a[1]);
    const int nl = *static_cast<int *>(a[2]);
    double *partials = *static_cast<double **>(a[3]);
    GridBarrier *bar = *static_cast<GridBarrier **>(a[4]);
    return std::function<void()>([=]() { scale_grid_kernel<T>(b, list, nl, partials, bar); });
  });
  return true;
}
const bool simt_bound = [] {
  using namespace osqpmi;
  ::simt::register_kernel((const void *)reset_counters_kernel, [](void **a) {
    int *c = *static_cast<int **>(a[0]);
    const int n = *static_cast<int *>(a[1]);
    GridBarrier *bar = *static_cast<GridBarrier **>(a[2]);
    return std::function<void()>([=]() { reset_counters_kernel(c, n, bar); });
  });
  return simt_bind_kernels<float>() && simt_bind_kernels<double>();
}();
}  // namespace
"""


HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
_RES_LINE = re.compile(r"remark:\s+(Function Name|VGPRs|AGPRs|LDS Size \[bytes/block\]):\s*(\S+)")


def gfx950_resources() -> dict:
    """Registers and static LDS of every kernel, as the gfx950 build of the
    library reports them (hipcc's kernel-resource-usage remarks, with the
    product build's code-generation flags): {(name, type): (vgpr, agpr, lds)},
    type 'f', 'd' or '' for a kernel that is not a template."""
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "--cuda-device-only", "-c", "-o", os.devnull, "-Rpass-analysis=kernel-resource-usage",
           os.path.join(CSRC, "api.hip")]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stderr[-4000:])
        raise RuntimeError("gfx950 resource report failed")
    out, cur = {}, None
    for line in res.stderr.splitlines():
        m = _RES_LINE.search(line)
        if not m:
            continue
        key, val = m.group(1), m.group(2)
        if key == "Function Name":
            mm = re.match(r"_ZN6osqpmi(\d+)", val)
            if not mm:
                cur = None
                continue
            ln = int(mm.group(1))
            rest = val[mm.end():]
            name, rest = rest[:ln], rest[ln:]
            typ = rest[1] if rest.startswith("I") and rest[1] in "fd" else ""
            cur = [name, typ, 0, 0, 0]
            out[(name, typ)] = cur
        elif cur is not None:
            idx = {"VGPRs": 2, "AGPRs": 3}.get(key, 4)
            cur[idx] = int(val)
    return {k: tuple(v[2:]) for k, v in out.items()}


def resource_registrations(res: dict) -> str:
    """C++ that registers each kernel's gfx950 resources with the stand-in
    runtime (its occupancy and static-LDS queries read them)."""
    ctype = {"f": "float", "d": "double"}
    lines = ["namespace {", "const bool simt_resources_registered = [] {", "  using namespace osqpmi;"]
    for (name, typ), (vg, ag, lds) in sorted(res.items()):
        fn = f"{name}<{ctype[typ]}>" if typ else name
        lines.append(f"  ::simt::register_resources((const void *){fn}, {vg}, {ag}, {lds});")
    lines += ["  return true;", "}();", "}  // namespace", ""]
    return "\n".join(lines)


def _sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    files = [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC))]
    files += [os.path.join(ROOT, "include", "osqp_mi.h"), os.path.abspath(__file__),
              os.path.join(HERE, "include", "hip", "hip_runtime.h")]
    for f in files:
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode() + fh.read())
    h.update(CLANG.encode() + str(SEPARATE_ARRAYS).encode() + str(WITH_SERVER).encode())
    h.update(os.environ.get("SIMT_CU_COUNT", "256").encode())
    return h.hexdigest()


def build(verbose: bool = False, force: bool = False) -> str:
    """Builds the host library unless one built from the same sources is
    there."""
    os.makedirs(OUT_DIR, exist_ok=True)
    stamp = os.path.join(OUT_DIR, "sources.sha256")
    digest = _sources_hash()
    if not force and os.path.exists(LIB) and os.path.exists(stamp):
        with open(stamp) as fh:
            if fh.read().strip() == digest:
                return LIB
    with open(os.path.join(CSRC, "api.hip")) as fh:
        src = translate(fh.read())
    res = gfx950_resources()
    if ("solve_wg_kernel", "f") not in res or ("polish_wg_kernel", "d") not in res:
        raise RuntimeError("resource report lacks the solve or polish kernels")
    src += resource_registrations(res)
    cpp = os.path.join(OUT_DIR, "api_simt.cpp")
    with open(cpp, "w") as fh:
        fh.write(src)
    tmp = LIB + ".tmp"
    cmd = [CLANG, "-std=c++17", "-O1", "-g", "-fPIC", "-shared",
           f"-DSIMT_CU_COUNT={int(os.environ.get('SIMT_CU_COUNT', '256'))}",
           "-fsanitize=address", "-fno-omit-frame-pointer",
           "-Wno-unknown-pragmas", "-Wno-unused-command-line-argument",
           "-I", os.path.join(HERE, "include"), "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, "-x", "c++", cpp, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("host build of the kernels failed")
    os.replace(tmp, LIB)
    with open(stamp, "w") as fh:
        fh.write(digest + "\n")
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, force="--force" in sys.argv))
