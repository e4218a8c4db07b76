"""CPU model of the volume labelling over 2 x 2 x 2 voxel blocks (k_vb_init,
k_vb_union and k_vb_flatten in vol.hip).

TEST INFRASTRUCTURE.  It follows the kernels' decisions block by block: the
block bits, the runs of a chunk of 64 blocks (blocks joined through their x
faces), the run tags of the touched blocks in the four earlier block rows,
the two skip rules (one union per touched run; none for a run the left
neighbour of the same run already touches) and the unions of run starts.
The unions themselves run sequentially (the partition a union-find reaches
does not depend on the order of its unions), so the model checks which
unions the kernels make, not the concurrency of making them.
"""
import numpy as np

CHUNK = 64


def face(oz, oy, ox):
    """Voxels (dz, dy, dx) of a block that can touch its neighbour at offset
    (oz, oy, ox): coordinate 0 towards -1, 1 towards +1, any along 0."""
    m = 0
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                if all(o == 0 or (o < 0) == (d == 0) for o, d in ((oz, dz), (oy, dy), (ox, dx))):
                    m |= 1 << (dz * 4 + dy * 2 + dx)
    return m


def block_bits(vol):
    D, S, W = vol.shape
    BZ, BY, BX = (D + 1) // 2, (S + 1) // 2, (W + 1) // 2
    pad = np.zeros((2 * BZ, 2 * BY, 2 * BX), np.int64)
    pad[:D, :S, :W] = vol
    bits = np.zeros((BZ, BY, BX), np.int64)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                bits |= pad[dz::2, dy::2, dx::2] << (dz * 4 + dy * 2 + dx)
    return bits


def runs_of_chunk(row_bits, cx):
    """Run-start lane of every lane of chunk cx of one block row, and whether
    each lane's block joins its left neighbour (lane > 0 only)."""
    BX = len(row_bits)
    lanes = range(CHUNK)
    bit = [row_bits[CHUNK * cx + l] if CHUNK * cx + l < BX else 0 for l in lanes]
    conn = [l > 0 and bool(bit[l] & face(0, 0, -1)) and bool(bit[l - 1] & face(0, 0, 1)) for l in lanes]
    run, start = [], 0
    for l in lanes:
        if bit[l] and not conn[l]:
            start = l
        run.append(start if any(bit[k] and not conn[k] for k in range(l + 1)) else l)
    return bit, conn, run


def label(vol):
    """Block parents after the three passes: parent[k] = root block id."""
    bits = block_bits(vol)
    BZ, BY, BX = bits.shape
    CX = (BX + CHUNK - 1) // CHUNK
    P = np.full(BZ * BY * BX, -1, np.int64)
    bid = lambda z, y, x: (z * BY + y) * BX + x
    # init
    for z in range(BZ):
        for y in range(BY):
            for cx in range(CX):
                bit, conn, run = runs_of_chunk(bits[z, y], cx)
                for l in range(CHUNK):
                    x = CHUNK * cx + l
                    if x < BX and bit[l]:
                        P[bid(z, y, x)] = bid(z, y, CHUNK * cx + run[l])

    def find(a):
        while P[a] != a:
            a = P[a]
        return a

    def unite(a, b):
        a, b = find(a), find(b)
        if a != b:
            P[max(a, b)] = min(a, b)

    def bits_at(z, y, x):
        if z < 0 or y < 0 or y >= BY or x < 0 or x >= BX:
            return 0
        return int(bits[z, y, x])

    for z in range(BZ):
        for y in range(BY):
            for cx in range(CX):
                bit, conn, run = runs_of_chunk(bits[z, y], cx)
                tags_of = {}
                for l in range(CHUNK):
                    x = CHUNK * cx + l
                    me = bid(z, y, CHUNK * cx + run[l]) if x < BX else None
                    b = bit[l]
                    if l == 0 and b and (b & face(0, 0, -1)) and (bits_at(z, y, x - 1) & face(0, 0, 1)):
                        unite(bid(z, y, x), bid(z, y, x) - 1)
                    for q, (oz, oy) in enumerate(((0, -1), (-1, -1), (-1, 0), (-1, 1))):
                        rz, ry = z + oz, y + oy
                        if rz < 0 or ry < 0 or ry >= BY:
                            tags_of[(q, l)] = [-1, -1, -1]
                            continue
                        rbit, rconn, rrun = runs_of_chunk(bits[rz, ry], cx)
                        t = []
                        for j, ox in enumerate((-1, 0, 1)):
                            nbits = bits_at(rz, ry, x + ox)
                            touch = bool(b & face(oz, oy, ox)) and bool(nbits & face(-oz, -oy, -ox))
                            if not touch:
                                t.append(-1)
                            elif ox < 0:
                                t.append(64 if l == 0 else rrun[l - 1])
                            elif ox > 0:
                                t.append(65 if l == 63 else rrun[l + 1])
                            else:
                                t.append(rrun[l])
                        if t[1] == t[0]:
                            t[1] = -1
                        if t[2] == t[0] or t[2] == t[1]:
                            t[2] = -1
                        tags_of[(q, l)] = list(t)
                        left = tags_of.get((q, l - 1), [-1, -1, -1]) if l > 0 else [-1, -1, -1]
                        row0 = bid(rz, ry, CHUNK * cx)
                        for tj in t:
                            if tj < 0 or (conn[l] and tj in left):
                                continue
                            other = row0 - 1 if tj == 64 else row0 + 64 if tj == 65 else row0 + tj
                            unite(me, other)
    # flatten
    for k in range(len(P)):
        if P[k] >= 0:
            P[k] = find(k)
    return bits, P


def voxel_labels(vol):
    """Each voxel's smallest voxel index of its component (the canonical
    labels of the labelling entry point), -1 for background."""
    D, S, W = vol.shape
    bits, P = label(vol)
    BZ, BY, BX = bits.shape
    out = np.full(vol.shape, -1, np.int64)
    canon = {}
    zz, yy, xx = np.nonzero(vol)
    for z, y, x in zip(zz, yy, xx):
        r = P[((z // 2) * BY + y // 2) * BX + x // 2]
        v = (z * S + y) * W + x
        canon[r] = min(canon.get(r, v), v)
    for z, y, x in zip(zz, yy, xx):
        out[z, y, x] = canon[P[((z // 2) * BY + y // 2) * BX + x // 2]]
    return out
