"""The native geometry planner (lbm_plan.cpp, plain C++) compiled with g++ on the host under
AddressSanitizer and UBSan: node-type codes and solid-neighbour bits of the dense and tiled
layouts against a brute-force recomputation (no GPU needed)."""
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
        if (tiled == 2) {
            lbm::plan::Fluid fl = lbm::plan::fluid_list(mask.data(), nx, ny);
            lbm::plan::IndirectCompact ic =
                lbm::plan::indirect_compact(fl, mask.data(), nx, ny, fl.n_fluid);
            for (long n = 0; n < fl.n_fluid; ++n) {
                std::printf("%d %d %u %u", fl.xy[2 * n], fl.xy[2 * n + 1], (unsigned)ic.info[n], ic.pk[n]);
                if (ic.info[n] & 0x100)
                    for (int i = 0; i < 8; ++i) std::printf(" %d", ic.edge[ic.pk[n] * 8 + i]);
                std::printf("\n");
            }
            return 0;
        }
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
            lbm::plan::Tiles t = lbm::plan::tiles16(mask.data(), nx, ny, tiled == 3);
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
    # host-only build under AddressSanitizer and UBSan: any out-of-bounds access or
    # undefined behaviour in the planner aborts the driver and fails the test
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I", CSRC, str(src),
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


def test_tiled_types_keep_all(planner):
    """The "tile" layout keeps every tile, the all-solid ones (solid codes throughout) too."""
    m = synthetic.random_mask(48, 32, seed=4, solid_fraction=0.3)
    m[:, 16:32] = 1
    compact = _run(planner, m, 0, True)
    full = _run(planner, m, 0, 3)
    assert len(compact) == 4 * 256 and len(full) == 6 * 256
    seen = {(x, y) for x, y, _, _ in full}
    assert len(seen) == 48 * 32
    for x, y, t, b in full:
        assert (t, b) == _expected(m, x, y), (x, y)


def _decode(rows):
    """Neighbour indices from the compact description, by the documented rule."""
    out = []
    for n, r in enumerate(rows):
        x, y, info, pk = r[:4]
        bits = info & 0xFF
        solid = lambda i: (bits >> (i - 1)) & 1
        if info & 0x100:
            src = list(r[4:12])
        else:
            dn = ((pk & 0xFFFF) ^ 0x8000) - 0x8000
            up = ((pk >> 16) ^ 0x8000) - 0x8000
            qd, qu = n + dn, n + up
            src = [None] * 8
            src[0] = n - 1          # dir 1: (x-1, y)
            src[2] = n + 1          # dir 3: (x+1, y)
            src[1] = qd             # dir 2: (x, y-1)
            src[4] = qd - 1         # dir 5: (x-1, y-1)
            src[5] = qd + (1 - solid(2))  # dir 6: (x+1, y-1)
            src[3] = qu             # dir 4: (x, y+1)
            src[7] = qu - 1         # dir 8: (x-1, y+1)
            src[6] = qu + (1 - solid(4))  # dir 7: (x+1, y+1)
        out.append([(-1 if solid(i) else src[i - 1]) for i in range(1, 9)])
    return out


@pytest.mark.parametrize("shape,frac", [((37, 23), 0.3), ((64, 40), 0.0), ((9, 7), 0.5)])
def test_indirect_compact(planner, shape, frac):
    import paper_2108_13241_amd as lbm
    nx, ny = shape
    m = synthetic.random_mask(nx, ny, seed=nx + 3 * ny, solid_fraction=frac)
    ny_, nx_ = m.shape
    inp = f"{nx} {ny} 0 2\n" + " ".join(str(int(v)) for v in m.ravel())
    r = subprocess.run([planner], input=inp, capture_output=True, text=True)
    assert r.returncode == 0
    rows = [list(map(int, ln.split())) for ln in r.stdout.split("\n") if ln.strip()]
    _, nbr = lbm.plan_indirect(m)  # plain table: nbr[i-1][n]
    dec = _decode(rows)
    assert len(dec) == nbr.shape[1]
    for n, d in enumerate(dec):
        assert d == list(nbr[:, n]), n
    # interior nodes use the compact form
    assert sum(1 for r in rows if not r[2] & 0x100) > 0


DRIVER3 = textwrap.dedent(r"""
    #include <cstdio>
    #include <vector>
    #include "lbm_plan.h"
    int main() {
        int nx, ny, nz, pitch;
        if (std::scanf("%d %d %d %d", &nx, &ny, &nz, &pitch) != 4) return 2;
        std::vector<uint8_t> mask((size_t)nx * ny * nz);
        for (auto &m : mask) { int v; if (std::scanf("%d", &v) != 1) return 2; m = (uint8_t)v; }
        std::vector<uint8_t> type;
        std::vector<uint32_t> nbits, seg;
        lbm::plan::dense_types3(mask.data(), nx, ny, nz, pitch, type, nbits, seg);
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < pitch; ++x) {
                    const size_t p = ((size_t)z * ny + y) * pitch + x;
                    std::printf("%d %u\n", type[p], nbits[p]);
                }
        for (uint32_t f : seg) std::printf("%u\n", f);
        return 0;
    }
""")


@pytest.fixture(scope="module")
def planner3(tmp_path_factory):
    d = tmp_path_factory.mktemp("plan3")
    src = d / "drv3.cpp"
    src.write_text(DRIVER3)
    exe = d / "drv3"
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I", CSRC, str(src),
                    os.path.join(CSRC, "lbm_plan.cpp"), "-o", str(exe)], check=True)
    return str(exe)


@pytest.mark.parametrize("shape", [(70, 9, 7), (300, 3, 2), (1, 1, 1), (1, 1, 5), (64, 2, 3)])
def test_dense_types3_brute_force(planner3, oracle_mod, shape):
    """D3Q19 node types, solid-neighbour bits (velocities from the pinned D3Q19 oracle) and
    256-node interior-segment flags, padding columns solid."""
    nx, ny, nz = shape
    pitch = (nx + 63) // 64 * 64
    m = synthetic.random_mask3(nx, ny, nz, seed=nx + 7 * ny + 13 * nz, solid_fraction=0.1)
    inp = f"{nx} {ny} {nz} {pitch}\n" + " ".join(str(int(v)) for v in m.ravel())
    r = subprocess.run([planner3], input=inp, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    rows = [list(map(int, ln.split())) for ln in r.stdout.split("\n") if ln.strip()]
    n_pad = nz * ny * pitch
    cells = np.array(rows[:n_pad]).reshape(nz, ny, pitch, 2)
    seg = np.array([v[0] for v in rows[n_pad:]])
    cx, cy, cz, _, _ = oracle_mod.constants3()
    bpr = (nx + 255) // 256
    exp_seg = np.ones(nz * ny * bpr, int)
    for z in range(nz):
        for y in range(ny):
            assert (cells[z, y, nx:, 0] == 1).all()
            for x in range(nx):
                t, b = cells[z, y, x]
                if m[z, y, x]:
                    assert t == 1
                else:
                    bits = 0
                    for i in range(1, 19):
                        if m[(z - cz[i]) % nz, (y - cy[i]) % ny, (x - cx[i]) % nx]:
                            bits |= 1 << (i - 1)
                    assert (t, b) == ((2 if bits else 0), bits)
                if t != 0:
                    exp_seg[(z * ny + y) * bpr + x // 256] = 0
    assert np.array_equal(seg, exp_seg)


DRIVER_LIST3 = textwrap.dedent(r"""
    #include <algorithm>
    #include <cstdio>
    #include <vector>
    #include "lbm_plan.h"
    int main() {
        int nx, ny, nz;
        if (std::scanf("%d %d %d", &nx, &ny, &nz) != 3) return 2;
        std::vector<uint8_t> mask((size_t)nx * ny * nz);
        for (auto &m : mask) { int v; if (std::scanf("%d", &v) != 1) return 2; m = (uint8_t)v; }
        long n_f = 0;
        for (auto m : mask) n_f += m == 0;
        const long np = std::max(64L, (n_f + 63) / 64 * 64);
        lbm::plan::Fluid3 fl = lbm::plan::fluid_list3(mask.data(), nx, ny, nz, np);
        const long ne = std::max<long>(fl.n_edge, 1);
        for (long n = 0; n < fl.n_fluid; ++n) {
            std::printf("%d %d %d %u", fl.xyz[3 * n], fl.xyz[3 * n + 1], fl.xyz[3 * n + 2],
                        fl.info[n]);
            for (int i = 0; i < 18; ++i) std::printf(" %d", fl.nbr[(size_t)i * np + n]);
            for (int r = 0; r < 8; ++r) std::printf(" %d", fl.rank8[(size_t)r * np + n]);
            if (fl.info[n] & lbm::plan::kListBorder)
                for (int i = 0; i < 18; ++i) std::printf(" %d", fl.edge[(size_t)i * ne + fl.rank8[n]]);
            std::printf("\n");
        }
        for (long n = fl.n_fluid; n < np; ++n)
            for (int i = 0; i < 18; ++i)
                if (fl.nbr[(size_t)i * np + n] != -1) return 3;
        return 0;
    }
""")

CX3 = [0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0]
CY3 = [0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1]
CZ3 = [0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1]
ROWS3 = [(-1, 0), (1, 0), (0, -1), (0, 1), (-1, -1), (1, -1), (-1, 1), (1, 1)]


def _decode_list3(n, info, rank8, edge):
    """Pull sources of list node n from the compact form, by the documented rule: a border
    node (bit 31) holds its slot in the border table in place of the row-0 rank and takes
    from that table the sources with c_x != 0 and the row-0 source; every other source comes
    from the rank arithmetic."""
    border = bool(info & (1 << 31))
    solid = lambda i: (info >> (i - 1)) & 1
    out = []
    for i in range(1, 19):
        if solid(i):
            out.append(-1)
            continue
        dx, dy, dz = -CX3[i], -CY3[i], -CZ3[i]
        if border and (dx != 0 or (dz == 0 and dy < 0)):
            out.append(edge[i - 1])
            continue
        if dy == 0 and dz == 0:
            out.append(n + dx)
            continue
        q = rank8[ROWS3.index((dy, dz))]
        if dx == 0:
            out.append(q)
        elif dx < 0:
            out.append(q - 1)
        else:  # x + 1 in that row: q plus one if (x, row) itself is fluid
            j = [k for k in range(1, 19) if (CX3[k], CY3[k], CZ3[k]) == (0, -dy, -dz)][0]
            out.append(q + (1 - solid(j)))
    return out


@pytest.fixture(scope="module")
def planner_list3(tmp_path_factory):
    d = tmp_path_factory.mktemp("plan_list3")
    src = d / "drv.cpp"
    src.write_text(DRIVER_LIST3)
    exe = d / "drv"
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I", CSRC, str(src),
                    os.path.join(CSRC, "lbm_plan.cpp"), "-o", str(exe)], check=True)
    return str(exe)


@pytest.mark.parametrize("shape,frac", [((13, 7, 5), 0.35), ((9, 6, 4), 0.0), ((5, 4, 3), 0.7),
                                        ((2, 3, 3), 0.3), ((1, 1, 1), 0.0), ((3, 1, 1), 0.0),
                                        ((6, 1, 2), 0.3), ((5, 2, 1), 0.2), ((1, 4, 3), 0.25),
                                        ((7, 3, 1), 0.3), ((4, 4, 4), 1.0)])
def test_fluid_list3(planner_list3, shape, frac):
    """The full source table against brute force; the compact form (solid bits, eight row
    ranks, border nodes through the edge table) decodes to the same table.  The small shapes
    are one or two nodes wide in some axis, where a node's neighbour rows coincide with its
    own row (or the wrap in x makes every node a border node)."""
    nx, ny, nz = shape
    m = synthetic.random_mask3(nx, ny, nz, seed=nx * ny + nz, solid_fraction=frac)
    inp = f"{nx} {ny} {nz}\n" + " ".join(str(int(v)) for v in m.ravel())
    r = subprocess.run([planner_list3], input=inp, capture_output=True, text=True)
    assert r.returncode == 0, r.returncode
    rows = [list(map(int, ln.split())) for ln in r.stdout.split("\n") if ln.strip()]
    fluid = [(x, y, z) for z in range(nz) for y in range(ny) for x in range(nx) if m[z, y, x] == 0]
    index = {p: k for k, p in enumerate(fluid)}
    assert len(rows) == len(fluid)
    border = 0
    for n, row in enumerate(rows):
        x, y, z, info = row[:4]
        assert (x, y, z) == fluid[n]
        nbr = row[4:22]
        for i in range(1, 19):
            src = ((x - CX3[i]) % nx, (y - CY3[i]) % ny, (z - CZ3[i]) % nz)
            assert nbr[i - 1] == index.get(src, -1), (n, i)
        border += bool(info & (1 << 31))
        assert _decode_list3(n, info, row[22:30], row[30:48]) == nbr, n
    if frac < 0.5 and nx > 2:
        assert 0 < border < len(rows)


DRIVER_BLOCKS3 = textwrap.dedent(r"""
    #include <cstdio>
    #include <vector>
    #include "lbm_plan.h"
    int main() {
        int nx, ny, nz, keep_all;
        if (std::scanf("%d %d %d %d", &nx, &ny, &nz, &keep_all) != 4) return 2;
        std::vector<uint8_t> mask((size_t)nx * ny * nz);
        for (auto &m : mask) { int v; if (std::scanf("%d", &v) != 1) return 2; m = (uint8_t)v; }
        lbm::plan::Blocks3 b = lbm::plan::blocks4(mask.data(), nx, ny, nz, keep_all != 0);
        if ((long)b.fluid.size() != b.n_blocks + 1 || b.fluid[b.n_blocks] != 0) return 3;
        std::printf("%ld\n", (long)b.n_blocks);
        for (long k = 0; k < b.n_blocks; ++k) {
            std::printf("%d %d %d", b.xyz[3 * k], b.xyz[3 * k + 1], b.xyz[3 * k + 2]);
            for (int w = 0; w < lbm::plan::kBlockMetaWords; ++w)
                std::printf(" %u", b.meta[(size_t)k * lbm::plan::kBlockMetaWords + w]);
            std::printf(" %llu\n", (unsigned long long)b.fluid[k]);
        }
        return 0;
    }
""")


@pytest.fixture(scope="module")
def planner_blocks3(tmp_path_factory):
    d = tmp_path_factory.mktemp("plan_blocks3")
    src = d / "drv.cpp"
    src.write_text(DRIVER_BLOCKS3)
    exe = d / "drv"
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I", CSRC, str(src),
                    os.path.join(CSRC, "lbm_plan.cpp"), "-o", str(exe)], check=True)
    return str(exe)


def _block_source(nb, k, l, i):
    """The step kernel's pull-source rule for slot l of block k, direction i: the block across
    the crossed faces (offset = -c_i on the crossed axes, a D3Q19 velocity) and the slot."""
    lx, ly, lz = l & 3, (l >> 2) & 3, l >> 4
    cx, cy, cz = CX3[i], CY3[i], CZ3[i]
    X = (cx > 0 and lx == 0) or (cx < 0 and lx == 3)
    Y = (cy > 0 and ly == 0) or (cy < 0 and ly == 3)
    Z = (cz > 0 and lz == 0) or (cz < 0 and lz == 3)
    off = (-cx if X else 0, -cy if Y else 0, -cz if Z else 0)
    b = k if off == (0, 0, 0) else nb[[(CX3[j], CY3[j], CZ3[j]) for j in range(19)].index(off)]
    slot = ((lx - cx) & 3) | (((ly - cy) & 3) << 2) | (((lz - cz) & 3) << 4)
    return b, slot


@pytest.mark.parametrize("shape,frac,keep_all", [((12, 8, 8), 0.3, False), ((8, 8, 4), 0.0, False),
                                                 ((4, 4, 4), 0.5, False), ((16, 4, 8), 0.6, True),
                                                 ((8, 12, 4), 1.0, False)])
def test_blocks4(planner_blocks3, shape, frac, keep_all):
    """D3Q19 4 x 4 x 4 block table against brute force: kept blocks (those with a fluid node,
    or all), block-neighbour indices (a dropped block reads as n_blocks), per-slot fluid bits,
    the all-fluid flag; and the step kernel's source rule applied to the table reaches, for
    every fluid node and direction, the node x - c_i (periodic) with the right solidity.
    Some shapes are one block wide in an axis, where a block is its own neighbour."""
    nx, ny, nz = shape
    m = synthetic.random_mask3(nx, ny, nz, seed=nx + 5 * ny + 11 * nz, solid_fraction=frac)
    if frac > 0 and frac < 1:
        m[:, :, 4:8] = 1  # whole solid blocks (dropped unless keep_all)
    inp = f"{nx} {ny} {nz} {int(keep_all)}\n" + " ".join(str(int(v)) for v in m.ravel())
    r = subprocess.run([planner_blocks3], input=inp, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.split("\n") if ln.strip()]
    nb_n = int(lines[0])
    rows = [list(map(int, ln.split())) for ln in lines[1:]]
    bx_n, by_n, bz_n = nx // 4, ny // 4, nz // 4
    blocks = [(bx, by, bz) for bz in range(bz_n) for by in range(by_n) for bx in range(bx_n)
              if keep_all or (m[4 * bz:4 * bz + 4, 4 * by:4 * by + 4, 4 * bx:4 * bx + 4] == 0).any()]
    assert nb_n == len(blocks) == len(rows)
    index = {b: k for k, b in enumerate(blocks)}
    fluid_bits = []
    for k, row in enumerate(rows):
        bx, by, bz = row[:3]
        assert (bx, by, bz) == blocks[k]
        bits = 0
        for l in range(64):
            if m[4 * bz + (l >> 4), 4 * by + ((l >> 2) & 3), 4 * bx + (l & 3)] == 0:
                bits |= 1 << l
        assert row[23] == bits
        fluid_bits.append(bits)
    fluid_bits.append(0)
    for k, row in enumerate(rows):
        bx, by, bz = row[:3]
        meta = row[3:23]
        for j in range(1, 19):
            nbk = ((bx + CX3[j]) % bx_n, (by + CY3[j]) % by_n, (bz + CZ3[j]) % bz_n)
            assert meta[j - 1] == index.get(nbk, nb_n), (k, j)
        interior = all(fluid_bits[e] == (1 << 64) - 1 for e in [k] + meta[:18])
        assert meta[18] == int(interior) and meta[19] == 0
        nb = [k] + meta[:18]
        for l in range(64):
            x, y, z = 4 * bx + (l & 3), 4 * by + ((l >> 2) & 3), 4 * bz + (l >> 4)
            if m[z, y, x]:
                continue
            for i in range(1, 19):
                b, slot = _block_source(nb, k, l, i)
                sx, sy, sz = (x - CX3[i]) % nx, (y - CY3[i]) % ny, (z - CZ3[i]) % nz
                solid = m[sz, sy, sx] == 1
                assert solid == (((fluid_bits[b] >> slot) & 1) == 0), (k, l, i)
                if not solid:
                    assert rows[b][:3] == [sx // 4, sy // 4, sz // 4], (k, l, i)
                    assert slot == (sx & 3) | ((sy & 3) << 2) | ((sz & 3) << 4)
