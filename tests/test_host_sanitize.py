"""The library's host-only computation, the Verlet buffer estimate (nb_buffer.cpp, Sec. V.B),
built with the host compiler's address and undefined-behaviour sanitizers and driven through
its C entry points over ordinary, coverage-table, rotating-class, degenerate and invalid
inputs: no sanitizer report, and every result equal to the product library's (hipcc build)
for the same call."""
import math
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# Two classes of a water-like system, a 2-type LJ table, a synthetic coverage table of
# 8 radii (cumulative pair counts: held[l][k] = all[k] for k <= l, beyond that a falling
# fraction of the shell), Ewald parameters.
DRIVER = r"""
#include <cmath>
#include <cstdio>
#include <vector>
#include "nb.h"

static nb_params params(int coulomb) {
    nb_params p = {};
    p.n_types = 2; p.coulomb = coulomb; p.modifier = NB_MOD_POTSHIFT;
    p.rc = 0.9f; p.rinner = 0.9f; p.rlist = 0.9f; p.eps_r = 1.f; p.eps_rf = INFINITY;
    p.ewald_beta = coulomb == NB_COUL_EWALD ? 3.47f : 0.f; p.epsfac = 138.935458f;
    p.nstlist = 40; p.nstprune = 1;
    return p;
}

int main() {
    const int64_t count[2] = {1000, 2000};
    const double mass[2] = {18.015, 18.015}, rot_len[2] = {0.0, 0.1}, rot_mass[2] = {0.0, 1.008};
    const float charge[2] = {-0.82f, 0.41f};
    const int32_t type[2] = {0, 1};
    const float lj[8] = {2.6e-3f, 2.6e-6f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const int n = 8;
    std::vector<float> R(n);
    std::vector<int64_t> all(n), cov((size_t)n * n);
    for (int k = 0; k < n; ++k) {
        R[k] = 0.9f + 0.02f * (float)k;
        all[k] = 1000 * (int64_t)(k + 1) * (k + 1) * (k + 1);
    }
    for (int l = 0; l < n; ++l)
        for (int k = 0; k < n; ++k)
            cov[(size_t)l * n + k] = k <= l ? all[k] : all[l] + (all[k] - all[l]) * 3 / (3 + (k - l));
    nb_buffer_input in = {};
    in.n_classes = 2; in.count = count; in.mass = mass; in.charge = charge; in.type = type;
    in.lj = lj; in.volume = 29.9; in.temperature = 300.0; in.dt = 0.002;
    for (int coulomb : {NB_COUL_RF, NB_COUL_EWALD, NB_COUL_NONE}) {
        const nb_params p = params(coulomb);
        for (int rot = 0; rot < 2; ++rot) {
            in.rot_len = rot ? rot_len : nullptr;
            in.rot_mass = rot ? rot_mass : nullptr;
            for (int steps : {1, 10, 40}) {
                for (double rl : {0.9, 0.95, 1.05}) {
                    double d = -1.0;
                    const int st = nb_buffer_drift(&p, &in, steps, rl, &d);
                    std::printf("drift %d %d %d %.3f %d %.17g\n", coulomb, rot, steps, rl, st, d);
                }
                double r = -1.0, d = -1.0;
                const int st = nb_buffer_estimate(&p, &in, steps, 0.005, 1.0, &r, &d);
                std::printf("estimate %d %d %d %d %.17g %.17g\n", coulomb, rot, steps, st, r, d);
            }
            // the cluster list of the coverage table
            in.n_cov = n; in.cov_radii = R.data(); in.covered = cov.data();
            for (int k = 0; k < n; ++k) {
                double d = -1.0;
                const int st = nb_buffer_drift(&p, &in, 40, (double)R[k], &d);
                std::printf("cdrift %d %d %d %d %.17g\n", coulomb, rot, k, st, d);
            }
            for (double tol : {1e-9, 5e-3, 1.0}) {
                double r = -1.0, d = -1.0;
                const int st = nb_buffer_estimate(&p, &in, 40, tol, 1.0, &r, &d);
                std::printf("cestimate %d %d %g %d %.17g %.17g\n", coulomb, rot, tol, st, r, d);
            }
            in.n_cov = 0; in.cov_radii = nullptr; in.covered = nullptr;
        }
    }
    // invalid input: each rejected with NB_ERR_ARG before anything is read past it
    const nb_params p = params(NB_COUL_EWALD);
    double d = 0.0, r = 0.0;
    std::printf("err %d", nb_buffer_drift(&p, nullptr, 40, 1.0, &d));
    std::printf(" %d", nb_buffer_drift(&p, &in, 0, 1.0, &d));
    std::printf(" %d", nb_buffer_drift(&p, &in, 40, 0.5, &d));
    std::printf(" %d", nb_buffer_drift(&p, &in, 40, 1.0, nullptr));
    std::printf(" %d", nb_buffer_estimate(&p, &in, 40, 0.0, 1.0, &r, &d));
    nb_buffer_input bad = in;
    bad.count = nullptr;
    std::printf(" %d", nb_buffer_drift(&p, &bad, 40, 1.0, &d));
    bad = in; bad.n_cov = 2; bad.cov_radii = nullptr;
    std::printf(" %d", nb_buffer_drift(&p, &bad, 40, 1.0, &d));
    bad = in; bad.n_cov = 8; bad.cov_radii = R.data(); bad.covered = cov.data();
    std::printf(" %d\n", nb_buffer_drift(&p, &bad, 40, 0.97, &d));   // radius not in the table
    return 0;
}
"""


@pytest.fixture(scope="module")
def driver_output(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    src, exe = d / "driver.cpp", d / "driver"
    src.write_text(DRIVER)
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "paper_2006_09167_amd", "csrc", "nb_buffer.cpp"),
                    str(src), "-o", str(exe)], check=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    return r.stdout.splitlines()


CLASSES = dict(count=[1000, 2000], mass=[18.015, 18.015], charge=[-0.82, 0.41], type=[0, 1])
ROT = dict(CLASSES, rot_len=[0.0, 0.1], rot_mass=[0.0, 1.008])
LJ = np.array([2.6e-3, 2.6e-6, 0, 0, 0, 0, 0, 0], np.float32).reshape(2, 2, 2)


def _coverage():
    n = 8
    R = np.float32(0.9) + np.float32(0.02) * np.arange(n, dtype=np.float32)
    all_ = 1000 * (np.arange(n, dtype=np.int64) + 1) ** 3
    cov = np.empty((n, n), np.int64)
    for l in range(n):
        for k in range(n):
            cov[l, k] = all_[k] if k <= l else all_[l] + (all_[k] - all_[l]) * 3 // (3 + k - l)
    return R, cov


def _params(api, coulomb):
    name = {0: "rf", 1: "ewald", 2: "none"}[coulomb]
    return api.make_params(2, name, rc=0.9, rinner=0.9, rlist=0.9,
                           beta=3.47 if name == "ewald" else 0.0, nstlist=40, nstprune=1)


def _status(fn):
    from paper_2006_09167_amd import api
    try:
        return 0, fn()
    except api.NBError as e:
        return e.status, None


def test_sanitized_buffer_estimate_matches_the_library(driver_output):
    from paper_2006_09167_amd import api
    R, cov = _coverage()
    checked = 0
    for line in driver_output:
        f = line.split()
        if f[0] == "err":
            continue
        coulomb, rot = int(f[1]), int(f[2])
        p, cls = _params(api, coulomb), (ROT if rot else CLASSES)
        if f[0] == "drift":
            steps, rl, st, d = int(f[3]), float(f[4]), int(f[5]), float(f[6])
            st2, d2 = _status(lambda: api.buffer_drift(p, cls, LJ, 29.9, 300.0, 0.002, steps, rl))
        elif f[0] == "estimate":
            steps, st, d = int(f[3]), int(f[4]), (float(f[5]), float(f[6]))
            st2, d2 = _status(lambda: api.buffer_estimate(p, cls, LJ, 29.9, 300.0, 0.002, steps,
                                                          0.005, 1.0))
        elif f[0] == "cdrift":
            k, st, d = int(f[3]), int(f[4]), float(f[5])
            st2, d2 = _status(lambda: api.buffer_drift(p, cls, LJ, 29.9, 300.0, 0.002, 40,
                                                       float(R[k]), coverage=(R, cov)))
        else:
            tol, st, d = float(f[3]), int(f[4]), (float(f[5]), float(f[6]))
            st2, d2 = _status(lambda: api.buffer_estimate(p, cls, LJ, 29.9, 300.0, 0.002, 40,
                                                          tol, 1.0, coverage=(R, cov)))
        assert st == st2, line
        if st == 0:
            assert np.allclose(d, d2, rtol=1e-12, atol=0.0), (line, d2)
            checked += 1
    assert checked >= 60
    # the outputs span the interesting cases: zero drift (steps = 1), positive drift, a
    # cluster estimate out of reach (NB_ERR_CAPACITY = 4) and one reached
    words = [l.split() for l in driver_output]
    assert any(w[0] == "drift" and w[3] == "1" and float(w[6]) == 0.0 for w in words)
    assert any(w[0] == "drift" and float(w[6]) > 0.0 for w in words)
    assert any(w[0] == "cestimate" and w[4] == "4" for w in words)
    assert any(w[0] == "cestimate" and w[4] == "0" for w in words)


def test_sanitized_buffer_estimate_rejects_invalid_input(driver_output):
    err = [l for l in driver_output if l.startswith("err")]
    assert err == ["err 1 1 1 1 1 1 1 1"]
