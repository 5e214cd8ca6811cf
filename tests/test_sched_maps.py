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


def _queue_snippets():
    fwd = _src("nb_forces.hip")
    pool = re.search(r"(const int p = g % kQueuePools;\n\s*const int runs_p = [^\n]*;)", fwd)
    done = re.search(r"(const int grp = \(int\)blockIdx\.x % kQueuePools;.*?groups - 1;)", fwd,
                     re.S)
    consts = re.search(r"(constexpr int kQueueStaticPermille.*?constexpr int kQueueWords[^\n]*)",
                       _src("nb_internal.h"), re.S)
    grid = re.search(r"if \(mode == kExecBalanced \|\| mode == kExecQueue\) grid = "
                     r"blocks\(d\.n_waves, kFwdWaves\);", fwd)
    dyn = re.search(r"\*dyn = queue \? \*waves \* kQueueDynPerTwoWaves / 2 : 0;",
                    open(os.path.join(CSRC, "nb_host.cpp")).read())
    assert pool and done and consts and grid and dyn, "queue-mode code not found"
    return pool.group(1), done.group(1), consts.group(1)


QUEUE_HOST = r"""
#include <algorithm>
#include <cstdio>
#include <random>
#include <vector>
using std::min;
constexpr int kFwdWaves = %(fwd)d;
%(consts)s
struct Dim3 { unsigned x; };
static Dim3 blockIdx, gridDim;
static int atomicAdd(int* p, int v) { const int o = *p; *p += v; return o; }

static void pool_of(int g, int n_dyn, int* pool, int* runs) {
%(pool)s
    *pool = p;
    *runs = runs_p;
}

static bool block_done(int* queue, int b) {
    blockIdx.x = b;
    bool s_last;
%(done)s
    return s_last;
}

static int fail(const char* what, int a, int b, int c) {
    std::printf("FAIL %%s %%d %%d %%d\n", what, a, b, c);
    return 1;
}

int main() {
    std::mt19937 rng(7);
    for (int n_waves = 1; n_waves <= 3000; n_waves += (n_waves < 300 ? 1 : 97)) {
        // the launch: one wavefront per own run, blocks of kFwdWaves; the dynamic runs
        const int grid = (n_waves + kFwdWaves - 1) / kFwdWaves, G = grid * kFwdWaves;
        const int n_dyn = n_waves * kQueueDynPerTwoWaves / 2;
        // every dynamic run is taken from exactly one pool that some wavefront draws from
        std::vector<int> taken(std::max(n_dyn, 1), 0), pool_seen(kQueuePools, 0);
        for (int g = 0; g < G; ++g) {
            int p, runs;
            pool_of(g, n_dyn, &p, &runs);
            if (p < 0 || p >= kQueuePools) return fail("pool range", n_waves, g, p);
            if (pool_seen[p]++) continue;                  // a pool's runs, counted once
            for (int t = 0; t < runs; ++t) {
                const int k = p + kQueuePools * t;
                if (k >= n_dyn || taken[k]++) return fail("run", n_waves, g, k);
            }
        }
        for (int k = 0; k < n_dyn; ++k)
            if (taken[k] != 1) return fail("run not taken", n_waves, k, n_dyn);
        // finishing blocks in any order: exactly the last one sees itself last, and the
        // counters it then clears are the only ones touched
        gridDim.x = grid;
        std::vector<int> queue(kQueueWords, 0), order(grid);
        for (int rep = 0; rep < 3; ++rep) {
            for (int b = 0; b < grid; ++b) order[b] = b;
            std::shuffle(order.begin(), order.end(), rng);
            for (int i = 0; i < grid; ++i)
                if (block_done(queue.data(), order[i]) != (i == grid - 1))
                    return fail("last block", n_waves, rep, i);
            for (int w = 0; w < kQueueWords; ++w) {
                const bool counter = (w >= kQueueDone && w < kQueueDone + kQueuePools * kPoolStride &&
                                      (w - kQueueDone) %% kPoolStride == 0) || w == kQueueDoneAll;
                if (!counter && queue[w] != 0) return fail("stray word", n_waves, rep, w);
            }
            // the last block's reset, as the kernel does it
            for (int k = 0; k < kQueuePools; ++k) queue[kQueueDone + k * kPoolStride] = 0;
            queue[kQueueDoneAll] = 0;
        }
    }
    std::printf("ok\n");
    return 0;
}
"""


@pytest.fixture(scope="module")
def queue_program(tmp_path_factory):
    pool, done, consts = _queue_snippets()
    text = QUEUE_HOST % dict(fwd=_const(_src("nb_forces.hip"), "kFwdWaves"), consts=consts,
                             pool=_indent(pool, 4), done=_indent(done, 4))
    d = tmp_path_factory.mktemp("queue")
    src, exe = d / "queue.cpp", d / "queue"
    src.write_text(text)
    subprocess.run(["g++", "-O1", "-std=c++17", "-Wall", "-Werror", "-o", str(exe), str(src)],
                   check=True, timeout=120)
    return str(exe)


def test_queue_runs_and_last_block_as_written_in_the_kernel(queue_program):
    r = subprocess.run([queue_program], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
