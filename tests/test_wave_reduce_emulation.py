"""Host emulation of the tile kernel's wave reduce-scatter and its
lane-to-output mapping (no GPU).

The VALU tile kernel sums NR per-lane values over the 64 lanes of a wave with
a butterfly reduce-scatter (`wave_reduce_scatter<N>` in csrc/apply.hip) and
the lanes then write the totals to (vector, row, re/im) outputs.  This test
takes that function's source text from apply.hip, compiles it for the host
with 64 threads standing in for the 64 lanes (a shuffle is a barrier-
synchronised exchange), and checks every total against a plain sum, for
N = 16, 32 and 64 and for both ways of choosing the kept half (selecting
values, and selecting array addresses).  Integer-valued inputs make every
sum exact, so the comparison is bitwise.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2606_31598_amd", "csrc", "apply.hip")

HARNESS = r"""
#include <barrier>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#define __device__
#define __forceinline__ inline
struct Idx { unsigned x; };
thread_local Idx threadIdx;
static std::barrier<>* g_bar;
static float g_slot[64];
static float __shfl_xor(float v, int mask)
{
    g_slot[threadIdx.x & 63] = v;
    g_bar->arrive_and_wait();
    const float r = g_slot[(threadIdx.x & 63) ^ mask];
    g_bar->arrive_and_wait();
    return r;
}

FUNCTION_SOURCE

// super_tile's mapping: NR = NV * RW * 2 values per lane, value index
// (v * RW + r) * 2 + comp; lanes with lane % G == 0, G = 64 / NR, write the
// total of index lane / G.
template <int NR>
static int run(int seed)
{
    std::vector<float> in(64 * NR), out(NR, -1.f), want(NR, 0.f);
    unsigned s = (unsigned)seed * 2654435761u + 1u;
    for (int k = 0; k < 64 * NR; ++k) {
        s = s * 1664525u + 1013904223u;
        in[k] = (float)((int)(s >> 20) - 2048);    // exact integers
    }
    for (int l = 0; l < 64; ++l)
        for (int q = 0; q < NR; ++q) want[q] += in[l * NR + q];
    std::barrier<> bar(64);
    g_bar = &bar;
    std::vector<std::thread> th;
    for (int l = 0; l < 64; ++l)
        th.emplace_back([&, l] {
            threadIdx.x = (unsigned)l;
            float v[NR];
            for (int q = 0; q < NR; ++q) v[q] = in[l * NR + q];
            const float tot = wave_reduce_scatter<NR>(v);
            constexpr int G = 64 / NR;
            if (l % G == 0) out[l / G] = tot;
            for (int g = 1; g < G; ++g)             // the lanes of one group agree
                if (l % G == g && tot != want[l / G]) std::abort();
        });
    for (auto& t : th) t.join();
    int bad = 0;
    for (int q = 0; q < NR; ++q) bad += out[q] != want[q];
    return bad;
}

int main()
{
    int bad = 0;
    for (int seed = 0; seed < 4; ++seed) bad += run<16>(seed) + run<32>(seed) + run<64>(seed);
    std::printf("mismatches %d\n", bad);
    return bad != 0;
}
"""


def _function_source():
    text = open(SRC).read()
    m = re.search(r"template <int N>\n__device__ __forceinline__ float wave_reduce_scatter"
                  r".*?\n}\n", text, re.S)
    assert m, "wave_reduce_scatter not found in apply.hip"
    return m.group(0)


@pytest.mark.parametrize("form", ["as_written", "values_everywhere", "addresses_everywhere"])
def test_wave_reduce_scatter_matches_plain_sum(tmp_path, form):
    if shutil.which("g++") is None:
        pytest.skip("no host C++ compiler")
    fn = _function_source()
    assert "if (N <= 32)" in fn
    if form == "values_everywhere":
        fn = fn.replace("if (N <= 32)", "if (true)")
    elif form == "addresses_everywhere":
        fn = fn.replace("if (N <= 32)", "if (false)")
    cpp = tmp_path / "emu.cpp"
    cpp.write_text(HARNESS.replace("FUNCTION_SOURCE", fn))
    exe = tmp_path / "emu"
    subprocess.run(["g++", "-std=c++20", "-O1", "-pthread", str(cpp), "-o", str(exe)],
                   check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "mismatches 0" in r.stdout
