"""Source text of device functions of the HIP kernels file, for host builds in CPU tests."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNELS = os.path.join(ROOT, "paper_2604_07170_amd", "csrc", "wfp2d_kernels.hip")
INTERNAL = os.path.join(ROOT, "paper_2604_07170_amd", "csrc", "wfp2d_internal.h")

# macros that let the kernels' device code compile as plain C++ (host threads stand in for
# a workgroup's lanes: threadIdx is per host thread, __syncthreads a barrier of the group)
HOST_PRELUDE = r"""
#include <barrier>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdio>
#include <random>
#include <thread>
#include <vector>
#define __device__
#define __global__
#define __forceinline__ inline
#define __shared__
#define __launch_bounds__(...)
struct float2 { float x, y; };
struct double2 { double x, y; };
inline float2 make_float2(float x, float y) { return float2{x, y}; }
inline double2 make_double2(double x, double y) { return double2{x, y}; }
struct HostDim { unsigned x, y; };
thread_local HostDim threadIdx;
HostDim blockIdx, blockDim;
std::barrier<> *host_group = nullptr;
inline void __syncthreads() { host_group->arrive_and_wait(); }
alignas(64) char smem[1 << 20];
"""


def definition(src: str, name: str) -> str:
    """Definition of `name` (with the bare template header line right above it, if any) up to
    its closing brace at column 0, or the one line it takes."""
    m = re.search(r"^(template <[^\n(]*\n)?(?!\s*//)[^\n]*\b" + re.escape(name) + r"(<[^>\n]*>)?\(", src, re.M)
    assert m, name
    start = m.start()
    first = src[start:src.index("\n", m.end())]
    if name == "from_d":                                   # declaration + two one-line specialisations
        end = src.index("from_d<double2>", start)
        return src[start:src.index("\n", end)]
    if first.rstrip().endswith("}"):
        return first
    return src[start:src.index("\n}\n", start) + 2]


def struct(src: str, name: str) -> str:
    i = src.index(f"struct {name} {{")
    return src[i:src.index("\n};\n", i) + 4]


def kernels_source() -> str:
    return open(KERNELS).read()


def internal_source() -> str:
    return open(INTERNAL).read()


def host_shared(text: str) -> str:
    """Workgroup-shared arrays as function statics (one workgroup runs at a time on the host);
    dynamic shared arrays stay extern globals of the harness."""
    text = text.replace("extern __shared__", "extern")
    return text.replace("__shared__", "static")


def between(src: str, start: str, end: str) -> str:
    """Source text from the line holding `start` up to (not including) the line holding `end`."""
    i = src.rindex("\n", 0, src.index(start)) + 1
    j = src.rindex("\n", 0, src.index(end, i)) + 1
    return src[i:j]
