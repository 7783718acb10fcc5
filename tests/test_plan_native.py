"""The native geometry planner (lbm_plan.cpp, plain C++) compiled with g++ on the host:
node-type codes and solid-neighbour bits of the dense and tiled layouts against a
brute-force recomputation (no GPU needed)."""
import os
import subprocess
import textwrap

import numpy as np
import pytest

import synthetic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2108_13241_amd", "csrc")

DRIVER = textwrap.dedent(r"""
    #include <cstdio>
    #include <vector>
    #include "lbm_plan.h"
    int main(int argc, char **argv) {
        int nx, ny, pitch, tiled;
        if (std::scanf("%d %d %d %d", &nx, &ny, &pitch, &tiled) != 4) return 2;
        std::vector<uint8_t> mask((size_t)nx * ny);
        for (auto &m : mask) { int v; if (std::scanf("%d", &v) != 1) return 2; m = (uint8_t)v; }
        std::vector<uint8_t> type, nmask;
        if (!tiled) {
            lbm::plan::dense_types(mask.data(), nx, ny, pitch, type, nmask);
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x)
                    std::printf("%d %d %d %d\n", x, y, type[(size_t)y * pitch + x],
                                nmask[(size_t)y * pitch + x]);
            for (int y = 0; y < ny; ++y)
                for (int x = nx; x < pitch; ++x)
                    if (type[(size_t)y * pitch + x] != 1) return 3;
        } else {
            lbm::plan::Tiles t = lbm::plan::tiles16(mask.data(), nx, ny);
            lbm::plan::tiled_types(mask.data(), nx, ny, t, type, nmask);
            for (long k = 0; k < t.n_tiles; ++k)
                for (int l = 0; l < 256; ++l)
                    std::printf("%d %d %d %d\n", t.xy[2 * k] * 16 + (l & 15),
                                t.xy[2 * k + 1] * 16 + (l >> 4), type[k * 256 + l],
                                nmask[k * 256 + l]);
        }
        return 0;
    }
""")


@pytest.fixture(scope="module")
def planner(tmp_path_factory):
    d = tmp_path_factory.mktemp("plan")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", CSRC, str(src),
                    os.path.join(CSRC, "lbm_plan.cpp"), "-o", str(exe)], check=True)
    return str(exe)


def _run(exe, m, pitch, tiled):
    ny, nx = m.shape
    inp = f"{nx} {ny} {pitch} {int(tiled)}\n" + " ".join(str(int(v)) for v in m.ravel())
    r = subprocess.run([exe], input=inp, capture_output=True, text=True)
    assert r.returncode == 0, r.returncode
    return np.array([list(map(int, ln.split())) for ln in r.stdout.split("\n") if ln.strip()])


def _expected(m, x, y):
    ny, nx = m.shape
    cx = [0, 1, 0, -1, 0, 1, -1, -1, 1]
    cy = [0, 0, 1, 0, -1, 1, 1, -1, -1]
    if m[y, x]:
        return 1, 0
    bits = 0
    for i in range(1, 9):
        if m[(y - cy[i]) % ny, (x - cx[i]) % nx]:
            bits |= 1 << (i - 1)
    return (2 if bits else 0), bits


@pytest.mark.parametrize("shape", [(37, 23), (64, 16), (5, 3)])
def test_dense_types(planner, shape):
    nx, ny = shape
    m = synthetic.random_mask(nx, ny, seed=nx * ny, solid_fraction=0.3)
    m[ny // 2, :] = 1
    rows = _run(planner, m, ((nx + 63) // 64) * 64, False)
    assert len(rows) == nx * ny
    for x, y, t, b in rows:
        assert (t, b) == _expected(m, x, y), (x, y)
    # every direction's bit occurs (the eighth one sits in the top bit of the byte)
    assert np.bitwise_or.reduce(rows[:, 3]) == 0xFF


def test_tiled_types(planner):
    m = synthetic.random_mask(48, 32, seed=4, solid_fraction=0.3)
    m[:, 16:32] = 1
    rows = _run(planner, m, 0, True)
    for x, y, t, b in rows:
        assert (t, b) == _expected(m, x, y), (x, y)
