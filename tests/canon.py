"""Independent checks of a message table (shared by oracle pins and GPU parity).

Nothing here re-implements the oracle's rectangle builder: the table is
checked against properties that characterise the canonical decomposition
uniquely (Sec. 4.2 "merging adjacent sections", made unique by the reading
recorded in the design notes):

  * coverage:    the boxes of destination d cover exactly the expected
                 element set E_d = {x in LUSE_d : d not a holder of x}, each
                 element once, and every element's source is its owner;
  * run maximality along the innermost dimension;
  * row stacking maximality inside a plane;
  * plane stacking maximality;
  * order:       (argument, lower corner row-major, destination), pack
                 offsets contiguous with element-size alignment.
"""
import numpy as np

F = dict(arg=0, array=1, src=2, dst=3, lo0=4, lo1=5, lo2=6, hi0=7, hi1=8, hi2=9, off=10, bytes=11)


def nshape(shape):
    return tuple([1] * (3 - len(shape)) + list(shape))


def box_slices(m):
    return (slice(m[4], m[7]), slice(m[5], m[8]), slice(m[6], m[9]))


def expected_sets(use_masks, owner, holders):
    """use_masks: dict dst -> bool array (nshape); owner/holders before the call.
    Returns dict dst -> int16 map (src, or -1)."""
    out = {}
    for d, m in use_masks.items():
        held = (holders >> np.uint64(d)) & np.uint64(1)
        need = m & (held == 0)
        e = np.full(m.shape, -1, dtype=np.int16)
        e[need] = owner[need]
        out[d] = e
    return out


def _run_is_maximal(row, c0, c1, s):
    """row: 1-D src map; [c0,c1) a maximal run of value s?"""
    if c1 <= c0 or not np.all(row[c0:c1] == s):
        return False
    if c0 > 0 and row[c0 - 1] == s:
        return False
    if c1 < row.shape[0] and row[c1] == s:
        return False
    return True


def check_array_messages(msgs, exp, esize=4):
    """msgs: rows of one array (any order as given); exp: dst -> src map.
    Raises AssertionError on the first violated property."""
    dsts = set(exp.keys()) | set(int(m[3]) for m in msgs)
    for d in dsts:
        e = exp.get(d)
        mine = [m for m in msgs if m[3] == d]
        if e is None:
            assert not mine, f"messages to {d} without a use region"
            continue
        cover = np.zeros(e.shape, dtype=np.int32)
        for m in mine:
            sl = box_slices(m)
            cover[sl] += 1
            blk = e[sl]
            assert blk.size > 0, f"empty box {m}"
            assert np.all(blk == m[2]), f"box {list(m)} has elements not sourced from {m[2]}"
        assert np.all(cover <= 1), f"overlapping boxes for dst {d}"
        assert np.array_equal(cover == 1, e >= 0), f"coverage mismatch for dst {d}"
        for m in mine:
            s, (p0, r0, c0, p1, r1, c1) = m[2], m[4:10]
            for p in range(p0, p1):
                for r in range(r0, r1):
                    assert _run_is_maximal(e[p, r], c0, c1, s), f"run not maximal {list(m)} at {(p, r)}"
            # row stacking: in plane p0 the row above/below must not carry the same maximal run
            for p in range(p0, p1):
                if r0 > 0:
                    assert not _run_is_maximal(e[p, r0 - 1], c0, c1, s), f"rows not stacked {list(m)}"
                if r1 < e.shape[1]:
                    assert not _run_is_maximal(e[p, r1], c0, c1, s), f"rows not stacked {list(m)}"

            # plane stacking: neighbouring plane must not carry the identical rectangle
            def has_rect(p):
                if p < 0 or p >= e.shape[0]:
                    return False
                for r in range(r0, r1):
                    if not _run_is_maximal(e[p, r], c0, c1, s):
                        return False
                if r0 > 0 and _run_is_maximal(e[p, r0 - 1], c0, c1, s):
                    return False
                if r1 < e.shape[1] and _run_is_maximal(e[p, r1], c0, c1, s):
                    return False
                return True

            assert not has_rect(p0 - 1) and not has_rect(p1), f"planes not stacked {list(m)}"


def check_order_and_offsets(msgs, esizes):
    """esizes: array id -> element size in bytes."""
    prev = None
    end = 0
    for m in msgs:
        key = (int(m[0]), int(m[4]), int(m[5]), int(m[6]), int(m[3]))
        if prev is not None:
            assert key > prev, f"messages out of order: {prev} then {key}"
        prev = key
        es = esizes[int(m[1])]
        off = (end + es - 1) // es * es
        assert m[10] == off, f"pack offset {m[10]} != {off}"
        vol = (m[7] - m[4]) * (m[8] - m[5]) * (m[9] - m[6])
        assert m[11] == vol * es
        end = off + m[11]
    return end


def pack_from_values(msgs, values_by_array):
    """Concatenate each message's box from the given array values (bytes)."""
    parts = []
    end = 0
    for m in msgs:
        v = values_by_array[int(m[1])]
        v3 = v.reshape(nshape(v.shape))
        es = v.dtype.itemsize
        off = (end + es - 1) // es * es
        if off > end:
            parts.append(np.zeros(off - end, dtype=np.uint8))
        blk = np.ascontiguousarray(v3[box_slices(m)])
        parts.append(blk.view(np.uint8).ravel())
        end = off + blk.nbytes
    return np.concatenate(parts) if parts else np.zeros(0, dtype=np.uint8)
