"""Host model of every buffer index the MDHP-LSTM kernels form (CPU only, no
library call): the GEMM calls of the forward and backward passes with their
strides, the split partials, the lane-packed copies of U, the recurrent
kernels' gate, cell, output and LDS indexes, and the saved-state and
workspace layouts, restated from mdhp_lstm.hip and checked against the
buffers' sizes for ragged and full shapes."""

import pytest

GT = 128
MAX_SPLIT = 64
ROWS = 16
XCDS = 8
FUSED_MAX_D = 256


def splits(Mr, Nc, Z, K):
    tiles = -(-Mr // GT) * -(-Nc // GT)
    s = -(-1024 // tiles)
    red = Z if Z > 1 else K // 256
    s = min(s, max(red, 1))
    return max(1, min(s, MAX_SPLIT))


def sizes(B, L, D, H, M, pair):
    Kb = M * M if pair else 1
    Kf = M * M + Kb + M
    saved = B * L * 5 * H + B * H + B * Kf
    part = max(MAX_SPLIT * max(4 * H * max(D, H), H * Kf), -(-B // ROWS) * 4 * H)
    Dp = -(-D // 16) * 16 if D <= FUSED_MAX_D else 0
    work = 8 * H * H + 4 * H * Dp + part + B * H
    return Kf, Kb, saved, part, work


def gemm_extent(base, saz, sai, sak, Z, Mr, K):
    """Largest element index A(z, i, k) can read (strides >= 0), or None."""
    if Z == 0 or Mr == 0 or K == 0:
        return None
    return base + (Z - 1) * saz + (Mr - 1) * sai + (K - 1) * sak


def check_gemm(name, A, B, C, Z, K, Mr, Nc, part_size, use_part):
    """A = (base, saz, sai, sak, size), B = (base, sbz, sbk, sbj, size),
    C = (ldc, size)."""
    a = gemm_extent(A[0], A[1], A[2], A[3], Z, Mr, K)
    b = gemm_extent(B[0], B[1], B[3], B[2], Z, Nc, K)
    if a is not None:
        assert a < A[4], (name, "A", a, A[4])
    if b is not None:
        assert b < B[4], (name, "B", b, B[4])
    if Mr and Nc:
        assert (Mr - 1) * C[0] + Nc - 1 < C[1], (name, "C")
    if use_part:
        S = splits(Mr, Nc, Z, K)
        assert S * Mr * Nc <= part_size, (name, "partials")


def model(B, L, D, H, M, pair):
    Kf, Kb, saved, part, work = sizes(B, L, D, H, M, pair)
    G, BL = 4 * H, B * L
    gates, cs_off, hks_off, feat_off = 0, BL * G, BL * G + BL * H, BL * G + BL * H + B * H
    assert feat_off + B * Kf == saved
    # forward: hks = tanh(feat Whks^T), gates = x W^T + b
    check_gemm("hks", (feat_off, 0, Kf, 1, saved), (0, 0, 1, Kf, H * Kf), (H, saved - hks_off),
               1, Kf, B, H, part, False)
    check_gemm("xproj", (0, 0, D, 1, BL * D), (0, 0, 1, D, G * D), (G, BL * G), 1, D, BL, G,
               part, False)
    # backward
    check_gemm("dx", (0, 0, G, 1, BL * G), (0, 0, D, 1, G * D), (D, BL * D), 1, G, BL, D,
               part, False)
    check_gemm("dW", (0, 0, 1, G, BL * G), (0, 0, D, 1, BL * D), (D, G * D), 1, BL, G, D,
               part, True)
    check_gemm("dU", (G, L * G, 1, G, BL * G), (0, L * H, H, 1, BL * H), (H, G * H), B, L - 1, G,
               H, part, True)
    check_gemm("dWhks", (0, 0, 1, H, B * H), (0, 0, Kf, 1, B * Kf), (Kf, H * Kf), 1, B, H, Kf,
               part, True)
    check_gemm("dfeat", (0, 0, H, 1, B * H), (0, 0, Kf, 1, H * Kf), (Kf, B * Kf), 1, H, B, Kf,
               part, False)
    # the bias gradient's per-workgroup column sums
    assert -(-B // ROWS) * G <= part
    # packed copies of U: H*H float4 each, indexes (nt KS + ks) 64 + lane
    KS, KT = H // 16, G // 16
    # the rows U rows / columns the packing reads
    assert 16 * (KS - 1) + 4 * 3 + 3 < H and 16 * (KT - 1) + 4 * 3 + 3 < G
    # recurrent kernels: H / 16 waves, wave w owns units 16 w .. 16 w + 15;
    # rows < B, t < L, col < 4H
    for wave in range(H // 16):
        u_max = 16 * wave + 15
        assert u_max < H and 3 * H + u_max < G
        for q in range(4):  # forward: Up[((q (H/16) + w) KS + ks) 64 + lane]
            assert ((q * (H // 16) + wave) * KS + KS - 1) * 64 + 63 < H * H
        assert ((wave * KT) + KT - 1) * 64 + 63 < H * H  # backward: UpT
    assert 4 * H <= 1024  # threads per workgroup
    if B:
        last = ((B - 1) * L + L - 1)
        assert last * G + G - 1 < BL * G and last * H + H - 1 < BL * H
    # LDS: float4 reads at row lr < 16, column 16 ks + 4 lq .. + 3
    HS, GS = H + 4, G + 4
    assert 15 * HS + 16 * (KS - 1) + 4 * 3 + 3 < ROWS * HS
    assert 15 * GS + 16 * (KT - 1) + 4 * 3 + 3 < ROWS * GS
    assert HS % 4 == 0 and GS % 4 == 0
    # fused forward recurrence (D <= 256): packed W of H * Dp float4 after
    # Up and UpT; float4 chunks of the x tile; LDS x tile [2][16][Dp + 4]
    Dp = -(-D // 16) * 16 if D <= FUSED_MAX_D else 0
    if Dp:
        KSD, QD, XS = Dp // 16, Dp // 4, Dp + 4
        for wave in range(H // 16):
            for q in range(4):
                assert ((q * (H // 16) + wave) * KSD + KSD - 1) * 64 + 63 < H * Dp
        for c in range(16 * QD):  # chunk c: row c // QD, features 4 (c % QD) ..
            row, d = divmod(c, QD)
            d *= 4
            n = min(max(D - d, 0), 4)
            assert row < 16 and d + 3 < XS and (n == 0 or d + n - 1 < D)
        assert 15 * XS + 4 * 3 + 16 * (KSD - 1) + 3 < 16 * XS
        assert 2 * 16 * XS * 4 <= 65536  # dynamic LDS of the x tile
        # the W packing reads columns k .. k + 3 only where k + s < D
    # workspace: Up, UpT, Wp, partials, dhks
    assert 8 * H * H + 4 * H * Dp + part + B * H == work


@pytest.mark.parametrize("B,L,D,H,M,pair", [
    (0, 3, 5, 64, 2, False), (1, 1, 1, 64, 1, False), (20, 7, 40, 64, 4, False),
    (37, 5, 33, 128, 3, True), (50, 9, 256, 256, 16, False), (4096, 128, 256, 256, 16, False),
    (4096, 128, 256, 256, 16, True), (100000, 2, 7, 128, 64, False)])
def test_lstm_indexes_in_bounds(B, L, D, H, M, pair):
    model(B, L, D, H, M, pair)


def test_split_partials_fit_for_every_gemm():
    for H in (64, 128, 256):
        for D in (1, 17, 256, 1024):
            for B in (1, 15, 16, 4096):
                model(B, 3, D, H, 8, False)


def gemm_tile(x, nJ, T):
    q, r = divmod(T, XCDS)
    xcd, slot = x % XCDS, x // XCDS
    t = xcd * (q + 1) + slot if xcd < r else r * (q + 1) + (xcd - r) * q + slot
    return divmod(t, nJ)


@pytest.mark.parametrize("nI,nJ", [(1, 1), (1, 3), (5, 2), (8, 2), (13, 7), (4096, 8)])
def test_gemm_tile_order_is_a_permutation(nI, nJ):
    T = nI * nJ
    seen = {gemm_tile(x, nJ, T) for x in range(T)}
    assert seen == {(i, j) for i in range(nI) for j in range(nJ)}
