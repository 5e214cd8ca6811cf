"""Block and wavefront index maps of the pair and backward kernels, checked on the host: the
XCD-contiguous renumbering of blocks and the persistent schedule's snake over the CU rounds
of blocks.  The code under test is cut out of the kernel sources as written and compiled
with the host compiler, so these checks follow every change to it."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2006_09167_amd", "csrc")


def _src(name):
    return open(os.path.join(CSRC, name)).read()


def _const(text, name):
    return int(re.search(r"constexpr int %s = (\d+);" % name, text).group(1))


def _xcd_block_body():
    m = re.search(r"__device__ inline int xcd_block\(int b, int g\) \{\n(.*?)\n\}\n",
                  _src("nb_forces.hip"), re.S)
    assert m, "xcd_block not found"
    return m.group(1)


def _snake(text, waves_name):
    """The persistent branch from the block's CU round to the item position of a round."""
    m = re.search(r"(const int b = \(int\)blockIdx\.x, r = b / n_cu.*?"
                  r"const int slot = base \+ \(odd \? G - 1 - g : g\);)", text, re.S)
    assert m, "persistent schedule not found"
    assert ("* %s + wave;" % waves_name) in m.group(1)
    return m.group(1)


HOST = r"""
#include <algorithm>
#include <cstdio>
#include <vector>
using std::min;
constexpr int kXcds = %(xcds)d;
constexpr int kFwdWaves = %(fwd)d;
constexpr int kBwdWaves = %(bwd)d;
struct Dim3 { unsigned x; };
static Dim3 blockIdx, gridDim;

static int xcd_block(int b, int g) {
%(xcd)s
}

// every (block, wavefront) of a persistent grid; visits[i] counts the wavefronts that
// take item i; pos_of[w] is the position of wavefront w (block * waves + wave)
static void fwd_persist(int n_cu, int grid, int n_items, std::vector<int>& visits,
                        std::vector<int>& pos_of) {
    const int G = grid * kFwdWaves;
    gridDim.x = grid;
    for (int blk = 0; blk < grid; ++blk)
        for (int wave = 0; wave < kFwdWaves; ++wave) {
            blockIdx.x = blk;
%(fwd_snake)s
                if (base == 0) pos_of[blk * kFwdWaves + wave] = g;
                if (slot < n_items) visits[slot]++;
            }
        }
}

static void bwd_persist(int n_cu, int grid, int n_items, std::vector<int>& visits,
                        std::vector<int>& pos_of) {
    const int G = grid * kBwdWaves;
    gridDim.x = grid;
    for (int blk = 0; blk < grid; ++blk)
        for (int wave = 0; wave < kBwdWaves; ++wave) {
            blockIdx.x = blk;
%(bwd_snake)s
                if (base == 0) pos_of[blk * kBwdWaves + wave] = g;
                if (slot < n_items) visits[slot]++;
            }
        }
}

static int fail(const char* what, int a, int b, int c) {
    std::printf("FAIL %%s %%d %%d %%d\n", what, a, b, c);
    return 1;
}

int main() {
    // XCD renumbering: a bijection on [0, g), and the blocks of one XCD (b mod kXcds)
    // take one contiguous range of positions, in block order
    for (int g = 1; g <= 5000; ++g) {
        std::vector<int> seen(g, 0);
        for (int b = 0; b < g; ++b) {
            const int v = xcd_block(b, g);
            if (v < 0 || v >= g || seen[v]++) return fail("xcd bijection", g, b, v);
            if (b >= kXcds && v != xcd_block(b - kXcds, g) + 1)
                return fail("xcd contiguous", g, b, v);
        }
    }
    // persistent rounds: every item taken exactly once, wavefront positions a bijection,
    // and odd CU rounds of blocks reversed
    const int cus[] = {1, 7, 256};
    for (int n_cu : cus)
        for (int grid = 1; grid <= 3 * n_cu + 5; grid += (n_cu > 8 ? 37 : 1))
            for (int n_items : {0, 1, grid * kFwdWaves - 1, grid * kFwdWaves,
                                 3 * grid * kFwdWaves + 5}) {
                for (int pass = 0; pass < 2; ++pass) {
                    const int waves = pass ? kBwdWaves : kFwdWaves;
                    std::vector<int> visits(std::max(n_items, 1), 0), pos(grid * waves, -1);
                    (pass ? bwd_persist : fwd_persist)(n_cu, grid, n_items, visits, pos);
                    for (int i = 0; i < n_items; ++i)
                        if (visits[i] != 1) return fail("item visits", n_cu, grid, i);
                    if (n_items == 0) continue;      // no round: no position taken
                    std::vector<int> seen(grid * waves, 0);
                    for (int w = 0; w < grid * waves; ++w) {
                        if (pos[w] < 0 || pos[w] >= grid * waves || seen[pos[w]]++)
                            return fail("position bijection", n_cu, grid, w);
                        const int blk = w / waves, r = blk / n_cu, at = blk %% n_cu;
                        const int m = std::min(n_cu, grid - r * n_cu);
                        const int want = r * n_cu + ((r %% 2) ? m - 1 - at : at);
                        if (pos[w] / waves != want) return fail("snake", n_cu, grid, w);
                    }
                }
            }
    std::printf("ok\n");
    return 0;
}
"""


def _indent(code, n):
    return "\n".join(" " * n + line.strip() for line in code.splitlines())


@pytest.fixture(scope="module")
def host_program(tmp_path_factory):
    fwd, bwd = _src("nb_forces.hip"), _src("nb_backward.hip")
    text = HOST % dict(
        xcds=_const(_src("nb_internal.h"), "kXcds"), fwd=_const(fwd, "kFwdWaves"),
        bwd=_const(bwd, "kBwdWaves"), xcd=_xcd_block_body(),
        fwd_snake=_indent(_snake(fwd, "kFwdWaves"), 12),
        bwd_snake=_indent(_snake(bwd, "kBwdWaves"), 12))
    d = tmp_path_factory.mktemp("sched")
    src, exe = d / "sched.cpp", d / "sched"
    src.write_text(text)
    subprocess.run(["g++", "-O1", "-std=c++17", "-Wall", "-Werror", "-o", str(exe), str(src)],
                   check=True, timeout=120)
    return str(exe)


def test_block_maps_as_written_in_the_kernels(host_program):
    r = subprocess.run([host_program], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
