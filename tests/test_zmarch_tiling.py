"""Host-side model of the z-marching sweeps' indexing (k_sweep_zm, load_plane,
zm_cell, PhiL in lbm_kernels.hpp; ztiles in lbm_api.hip): the tiles cover
every fluid cell exactly once, every halo load and LDS read stays in bounds,
and the LDS value a cell reads at offset (dx, dy, dz) is the phase field the
one-cell-per-thread stencil reads there (periodic x and z, periodic y or the
wall mirror onto the current row)."""
import itertools

import numpy as np
import pytest
kTX, kTY, kB, kZmBlocks = 64, 4, 256, 8192
kLX, kLY = kTX + 2, kTY + 2

def ztiles(nx, ny, nz):
    tx, ty = -(-nx // kTX), -(-ny // kTY)
    zc = max(1, min(64, tx * ty * nz // kZmBlocks))
    return tx, ty, -(-nz // zc), zc

def offm_cell(nx, ny, nz, walls, x, y, z, dx, dy, dz):
    xx = (x + dx) % nx
    if walls:
        yy = y + dy
        if dy < 0 and y == 1: yy = y
        if dy > 0 and y == ny - 2: yy = y
    else:
        yy = (y + dy) % ny
    zz = (z + dz) % nz
    return xx + nx * (yy + ny * zz)

def check(nx, ny, nz, walls):
    N = nx * ny * nz
    phi = np.arange(N, dtype=np.int64)       # value = its own index
    tx, ty, tz, zc = ztiles(nx, ny, nz)
    seen = np.zeros(N, dtype=np.int64)
    for b in range(tx * ty * tz):
        bx, r = b % tx, b // tx
        by, bz = r % ty, r // ty
        x0, y0, z0 = bx * kTX, by * kTY, bz * zc
        z1 = min(z0 + zc, nz)
        def plane(z):
            zz = z % nz
            buf = np.empty(kLX * kLY, dtype=np.int64)
            for i in range(kLX * kLY):
                hx, hy = i % kLX, i // kLX
                gx = (x0 - 1 + hx) % nx
                gy = y0 - 1 + hy
                gy = min(max(gy, 1), ny - 2) if walls else gy % ny
                g = gx + nx * (gy + ny * zz)
                assert 0 <= g < N
                buf[i] = phi[g]
            return buf
        pl = {z0 - 1: plane(z0 - 1), z0: plane(z0)}
        for z in range(z0, z1):
            pl[z + 1] = plane(z + 1)
            for t in range(kB):
                x, y = x0 + t % kTX, y0 + t // kTX
                active = x < nx and y < ny and not (walls and (y == 0 or y == ny - 1))
                o = (t // kTX + 1) * kLX + t % kTX + 1
                if not active:
                    continue
                c = x + nx * (y + ny * z)
                seen[c] += 1
                for dx, dy, dz in itertools.product((-1, 0, 1), repeat=3):
                    li = o + dy * kLX + dx
                    assert 0 <= li < kLX * kLY
                    assert pl[z + dz][li] == phi[offm_cell(nx, ny, nz, walls, x, y, z, dx, dy, dz)], (nx, ny, nz, walls, x, y, z, dx, dy, dz)
            del pl[z - 1]
    fluid = np.ones((nz, ny, nx), bool)
    if walls:
        fluid[:, 0, :] = fluid[:, -1, :] = False
    assert np.array_equal(seen.reshape(nz, ny, nx), fluid.astype(np.int64)), (nx, ny, nz, walls)



@pytest.mark.parametrize("shape", [(13, 21, 9, True), (16, 16, 16, False), (1, 18, 1, True), (12, 3, 10, True),
                                   (2, 2, 2, False), (1, 1, 1, False), (70, 9, 5, True), (64, 8, 3, False)])
def test_zmarch_tiles_reproduce_the_stencil(shape):
    check(*shape)


def test_zmarch_tiling_of_the_workloads():
    for (nx, ny, nz), blocks, zc in [((512, 512, 512), 8192, 64), ((128, 512, 128), 8192, 4),
                                      ((256, 1024, 256), 8192, 32)]:
        tx, ty, tz, c = ztiles(nx, ny, nz)
        assert tx * ty * tz == blocks and c == zc
