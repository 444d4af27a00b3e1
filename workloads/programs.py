"""HDArray programs of the workloads, written once and run on both the
oracle and the HIP runtime (the sequences of Table 2 calls a workload makes:
arrays, partitions, offsets and sections; no communication sets, no
kernels).  Both sides expose create / partition / kernel / set_offsets /
set_absolute / set_trapezoid / apply / write / read / reduce / messages /
pack / gdef with the same meaning).  Builtin ids: 1 jacobi2d, 2 copy,
3 matmul, 4 tri2d, 5 stencil3d7, 6 conv2d9; kinds: 0 ROW, 1 COL, 2 BLOCK."""
import numpy as np

ROW, COL, BLOCK = 0, 1, 2
K_JACOBI2D, K_COPY, K_MATMUL, K_TRI2D, K_STENCIL3D7, K_CONV2D9 = 1, 2, 3, 4, 5, 6
S3D_OFFSETS = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
J2D_OFFSETS = [(0, 0), (0, -1), (0, 1), (-1, 0), (1, 0)]


def jacobi_rows(api, A0, B0, ndev=4):
    """Jacobi with absolute use = own rows +-1 halo row, def = own rows
    (jacobi_small workload); two kernels for the ping-pong."""
    n0, n1 = A0.shape
    A, B = api.create(A0), api.create(B0)
    p = api.partition(ROW, (n0, n1), ndev=ndev)
    for k in ("jacAB", "jacBA"):
        api.kernel(k, K_JACOBI2D)
    for d in range(ndev):
        (_, r0, _), (_, r1, _) = api.part_region(p, d)
        if r0 >= r1:
            continue
        for k, out, inp in (("jacAB", A, B), ("jacBA", B, A)):
            api.set_absolute(k, p, inp, d, 0, (max(r0 - 1, 0), 0), (min(r1 + 1, n0), n1))
            api.set_absolute(k, p, out, d, 1, (r0, 0), (r1, n1))
    api.write(A, A0, p)
    api.write(B, B0, p)
    return A, B, p


def jacobi_blocks(api, A0, B0, ndev=16, use_box=False, kind=BLOCK):
    """Jacobi with a BLOCK partition (or another kind) and 5-point offsets
    (jacobi_large workload), or a full-box absolute use."""
    n0, n1 = A0.shape
    A, B = api.create(A0), api.create(B0)
    p = api.partition(kind, (n0, n1), ndev=ndev)
    for k, out, inp in (("jacAB", A, B), ("jacBA", B, A)):
        api.kernel(k, K_JACOBI2D)
        if use_box:
            for d in range(ndev):
                (_, r0, c0), (_, r1, c1) = api.part_region(p, d)
                api.set_absolute(k, p, inp, d, 0, (max(r0 - 1, 0), max(c0 - 1, 0)), (min(r1 + 1, n0), min(c1 + 1, n1)))
                api.set_absolute(k, p, out, d, 1, (r0, c0), (r1, c1))
        else:
            api.set_offsets(k, 1, 0, J2D_OFFSETS)
            api.set_offsets(k, 0, 1, [(0, 0)])
    api.write(A, A0, p)
    api.write(B, B0, p)
    return A, B, p


def gemm(api, a0, b0, P, layout=ROW):
    """Listings 2-3: use(A,(0,*)) use(B,(*,0)) def(C,(0,0))."""
    n, m = a0.shape[0], b0.shape[1]
    A, B, Cc = api.create(a0), api.create(b0), api.create(shape=(n, m))
    p = api.partition(layout, (n, m), ndev=P)
    api.kernel("gemm", K_MATMUL)
    api.set_offsets("gemm", 0, 0, [(0, "*")])
    api.set_offsets("gemm", 1, 0, [("*", 0)])
    api.set_offsets("gemm", 2, 1, [(0, 0)])
    pa = api.partition(layout, a0.shape, ndev=P)
    pb = api.partition(layout, b0.shape, ndev=P)
    api.write(A, a0, pa)
    api.write(B, b0, pb)
    return A, B, Cc, p


def tri(api, A0, B0, cuts):
    """Lower-triangular stencil on irregular row splits, trapezoid use/def."""
    n = A0.shape[0]
    nd = len(cuts) - 1
    A, B = api.create(A0), api.create(B0)
    p = api.partition_manual([(cuts[d], 0) for d in range(nd)], [(cuts[d + 1], n) for d in range(nd)])
    for k, out, inp in (("triAB", A, B), ("triBA", B, A)):
        api.kernel(k, K_TRI2D)
        for d in range(nd):
            a, b = cuts[d], cuts[d + 1]
            api.set_trapezoid(k, p, inp, d, 0, [a - 1, 0, a - 1, a - 1, b, 0, b, b])
            api.set_trapezoid(k, p, out, d, 1, [a, 0, a, a, b - 1, 0, b - 1, b - 1])
    api.write(A, A0, p)
    api.write(B, B0, p)
    return A, B, p


def stencil3d(api, u0, ndev=8):
    n = u0.shape
    U, V = api.create(np.zeros_like(u0)), api.create(u0)
    p = api.partition(BLOCK, n, ndev=ndev)
    for k, out, inp in (("s3dUV", U, V), ("s3dVU", V, U)):
        api.kernel(k, K_STENCIL3D7)
        api.set_offsets(k, 1, 0, S3D_OFFSETS)
        api.set_offsets(k, 0, 1, [(0, 0, 0)])
    api.write(U, np.zeros_like(u0), p)
    api.write(V, u0, p)
    return U, V, p


def batched_arrays(api, inst, seed=4):
    """The batched workload: per array either the 5-point Jacobi with use
    offsets (0,0),(0,+-1),(+-1,0) on irregular row splits, or the
    lower-triangular stencil with trapezoid use / def sections.  Kernels
    'b{i}AB' (A <- J(B)) and 'b{i}BA'.  Returns [(A, B, part, kind)]."""
    from workloads import batched_values
    out = []
    for m in inst:
        i, (H, W) = m["index"], m["shape"]
        A0, B0 = batched_values(seed, i, (H, W))
        A, B = api.create(A0), api.create(B0)
        cuts = [0] + [int(c) for c in m["cuts"]] + [H]
        nd = len(cuts) - 1
        p = api.partition_manual([(cuts[d], 0) for d in range(nd)], [(cuts[d + 1], W) for d in range(nd)])
        for k, o, s in ((f"b{i}AB", A, B), (f"b{i}BA", B, A)):
            if m["kind"] == 0:
                api.kernel(k, K_JACOBI2D)
                api.set_offsets(k, 1, 0, J2D_OFFSETS)
                api.set_offsets(k, 0, 1, [(0, 0)])
            else:
                api.kernel(k, K_TRI2D)
                for d in range(nd):
                    a, b = cuts[d], cuts[d + 1]
                    api.set_trapezoid(k, p, s, d, 0, [a - 1, 0, a - 1, a - 1, b, 0, b, b])
                    api.set_trapezoid(k, p, o, d, 1, [a, 0, a, a, b - 1, 0, b - 1, b - 1])
        api.write(A, A0, p)
        api.write(B, B0, p)
        out.append((A, B, p, m["kind"]))
    return out


def mm2(api, a0, b0, c0, P, layout=ROW):
    """Sec. 5.1 2MM: D = A x B, then E = C x D, both with the GEMM clauses
    use(X,(0,*)) use(Y,(*,0)) def(Z,(0,0)); ROW or COL partitions of the
    n x n work region (the partition argument is the only change)."""
    n = a0.shape[0]
    A, B, Cm = api.create(a0), api.create(b0), api.create(c0)
    D, E = api.create(shape=(n, n)), api.create(shape=(n, n))
    p = api.partition(layout, (n, n), ndev=P)
    for k in ("mm1", "mm2"):
        api.kernel(k, K_MATMUL)
        api.set_offsets(k, 0, 0, [(0, "*")])
        api.set_offsets(k, 1, 0, [("*", 0)])
        api.set_offsets(k, 2, 1, [(0, 0)])
    for X, x0 in ((A, a0), (B, b0), (Cm, c0)):
        api.write(X, x0, p)
    return A, B, Cm, D, E, p


CONV_OFFSETS = [(di, dj) for di in (-1, 0, 1) for dj in (-1, 0, 1)]


def conv2d(api, f0, ndev=16, kind=BLOCK):
    """Sec. 5.1 Convolution: 3 x 3 window (the eight neighbours and the
    centre) as use offsets, def = own block; convAB reads B into A, convBA
    reads A into B."""
    n0, n1 = f0.shape
    A, B = api.create(np.zeros_like(f0)), api.create(f0)
    p = api.partition(kind, (n0, n1), ndev=ndev)
    for k in ("convAB", "convBA"):
        api.kernel(k, K_CONV2D9)
        api.set_offsets(k, 1, 0, CONV_OFFSETS)
        api.set_offsets(k, 0, 1, [(0, 0)])
    api.write(A, np.zeros_like(f0), p)
    api.write(B, f0, p)
    return A, B, p
