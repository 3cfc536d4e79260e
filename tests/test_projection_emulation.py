"""CPU restatement of the branch-free basis loads of the fused sweeps (no GPU).

The fused projection of a staged batch of rows (SpMV + first CGS2 pass, and
the one-reduction SpMV + reduction) issues every basis-column load of a row
group unconditionally, in batches: a column past C -- or the SCALED kernel's
column j, whose values come from the staged v_j -- reads column 0 of the same
rows, and rows past the batch are masked by bit after the load.  The fp32
update + projection, one step at a time, lets a lane past the block's rows
load the step's first row and keeps only the wave-uniform column test as a
branch.

Checked here, for aligned batches with ragged ends, every column class and
both batch sizes: every load stays inside its basis column's padded length;
with NaN in the padded rows past n and stale NaN in the staged rows past the
batch (the row-tiled kernel does not clear them), each lane's partial sums
equal, bit for bit, those of the branch-per-load form the kernels had before;
and their total matches V^T y in fp64.  The update step's w' is checked the
same way against a direct evaluation.
"""
import numpy as np
import pytest

WAVE = 64
f32 = np.float32


def basis(n, ldv, ncols, rng):
    V = np.full((ncols, ldv), np.nan, f32)
    V[:, :n] = rng.uniform(-1, 1, (ncols, n))
    return V


def project_branchy(V, j, C, base, nrows, ys, vs, slots, nw, G, scaled):
    """The earlier form: each column's load under its own branch."""
    acc = np.zeros((nw, WAVE, slots), f32)
    ngroups = -(-nrows // G)
    for wid in range(nw):
        for lane in range(WAVE):
            for g in range(lane, ngroups, WAVE):
                rb = g * G
                yv = [ys[rb + i] if rb + i < nrows else f32(0) for i in range(G)]
                for q in range(slots):
                    c = wid + nw * q
                    if c >= C:
                        continue
                    if scaled and c == j:
                        vv = [vs[rb + i] if rb + i < nrows else f32(0) for i in range(G)]
                    else:
                        vv = [V[c, base + rb + i] if rb + i < nrows else f32(0) for i in range(G)]
                    s = acc[wid, lane, q]
                    for i in range(G):
                        s = f32(s + f32(vv[i] * yv[i]))
                    acc[wid, lane, q] = s
    return acc


def zero_unless(x, keep):
    return x if keep else f32(0)  # a bit mask: +0 whatever x holds (NaN included)


def project_batched(V, ldv, j, C, base, nrows, ys, vs, slots, nw, G, pq, scaled):
    """The branch-free form, with every load's address checked."""
    ncols = V.shape[0]
    acc = np.zeros((nw, WAVE, slots), f32)
    ngroups = -(-nrows // G)
    qb = min(slots, pq)
    assert base % G == 0
    for wid in range(nw):
        for lane in range(WAVE):
            for g in range(lane, ngroups, WAVE):
                rb = g * G
                assert rb + G <= len(ys)  # staged vectors hold the whole stage
                yv = [zero_unless(ys[rb + i], rb + i < nrows) for i in range(G)]
                for q0 in range(0, slots, qb):
                    raw = []
                    for u in range(qb):
                        c = wid + nw * (q0 + u)
                        from_v = c < C and not (scaled and c == j)
                        col = c if from_v else 0
                        assert 0 <= col < ncols
                        assert base + rb + G <= ldv, (base, rb, ldv)
                        raw.append(V[col, base + rb:base + rb + G].copy())
                    for u in range(qb):
                        c = wid + nw * (q0 + u)
                        if c >= C:
                            continue
                        if scaled and c == j:
                            vv = [zero_unless(vs[rb + i], rb + i < nrows) for i in range(G)]
                        else:
                            vv = [zero_unless(raw[u][i], rb + i < nrows) for i in range(G)]
                        s = acc[wid, lane, q0 + u]
                        for i in range(G):
                            s = f32(s + f32(vv[i] * yv[i]))
                        acc[wid, lane, q0 + u] = s
    return acc


@pytest.mark.parametrize("n,stage,base_frac,C,slots,nw,G,pq,scaled", [
    (3000, 1024, 0, 9, 2, 8, 4, 4, True),      # narrow class, SCALED, full stage
    (3000, 1024, 2, 30, 4, 8, 4, 4, True),     # last stage ragged (3000 - 2048 rows)
    (2100, 1024, 2, 50, 8, 8, 4, 4, False),    # 52 rows left, non-SCALED
    (1500, 512, 2, 100, 16, 8, 4, 4, True),    # wide class, C past half the slots
    (1500, 512, 2, 100, 16, 8, 4, 8, False),   # the one-reduction batch size
    (1100, 1024, 1, 33, 8, 8, 8, 4, True),     # bf16 row groups of 8, 76 rows left
    (2049, 1024, 2, 16, 4, 4, 4, 4, True),     # one row in the last stage
])
def test_batched_projection_matches_branchy(n, stage, base_frac, C, slots, nw, G, pq, scaled):
    assert C <= nw * slots  # the kernels cap C at the columns their slots hold
    rng = np.random.default_rng(n + C)
    ldv = -(-n // 128) * 128
    m = max(C, nw * slots) + 1
    V = basis(n, ldv, m, rng)
    base = base_frac * stage
    nrows = min(stage, n - base)
    j = C - 1
    ys = np.full(stage, np.nan, f32)  # stale rows past the batch, as in the tiled kernel
    vs = np.full(stage, np.nan, f32)
    ys[:nrows] = rng.uniform(-1, 1, nrows)
    vs[:nrows] = V[j, base:base + nrows] if not scaled else rng.uniform(-1, 1, nrows)
    a = project_batched(V, ldv, j, C, base, nrows, ys, vs, slots, nw, G, pq, scaled)
    b = project_branchy(V, j, C, base, nrows, ys, vs, slots, nw, G, scaled)
    assert np.all(np.isfinite(a))
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    # the total per column against V^T y in fp64
    tot = np.zeros(m)
    for wid in range(nw):
        for q in range(slots):
            c = wid + nw * q
            if c < C:
                tot[c] = a[wid, :, q].astype(np.float64).sum()
    Vd = V[:, base:base + nrows].astype(np.float64)
    if scaled:
        Vd[j] = vs[:nrows]
    ref = Vd[:C] @ ys[:nrows].astype(np.float64)
    assert np.allclose(tot[:C], ref, rtol=1e-5, atol=1e-4)


def update_step_fp32(n, k, slots, B, WV, R=4, seed=0):
    """One-step-at-a-time fp32 update + projection: w' = w - V h, V^T w'."""
    STEP = WAVE * R
    rng = np.random.default_rng(seed)
    ldv = -(-n // 128) * 128
    V = basis(n, ldv, k + 1, rng)
    w = np.full(ldv, np.nan, f32)
    w[:n] = rng.uniform(-1, 1, n)
    h = np.zeros(WV * slots, f32)
    h[:k] = rng.uniform(-1, 1, k)
    out = np.full(ldv, np.nan, f32)
    written = np.zeros(n, int)
    acc = np.zeros(WV * slots)
    for b in range(B):
        chunk = -(-n // B)
        chunk = (chunk + 63) & ~63
        r0, r1 = min(b * chunk, n), min(b * chunk + chunk, n)
        for base in range(r0, r1, STEP):
            part = np.zeros((WV, WAVE, R), f32)
            vals = {}
            for wid in range(WV):
                for lane in range(WAVE):
                    r = base + R * lane
                    nv = r1 - r
                    s = [f32(0)] * R
                    for q in range(slots):
                        c = wid + WV * q
                        if c < k:  # the only branch: wave-uniform
                            row = r if nv > 0 else base
                            assert 0 <= row and row + R <= ldv
                            v = V[c, row:row + R].copy()
                        else:
                            v = np.zeros(R, f32)
                        vals[(wid, lane, q)] = v
                        for i in range(R):
                            s[i] = f32(s[i] + f32(h[c] * (v[i] if i < nv else f32(0))))
                    part[wid, lane] = s
            for lane in range(WAVE):
                r = base + R * lane
                nv = r1 - r
                row = r if nv > 0 else base
                assert row + R <= ldv
                wv = w[row:row + R].copy()
                t = [f32(f32(part[0, lane, i] + part[1, lane, i]) + f32(part[2, lane, i] + part[3, lane, i])) for i in range(R)]
                if WV == 8:
                    t = [f32(t[i] + f32(f32(part[4, lane, i] + part[5, lane, i]) + f32(part[6, lane, i] + part[7, lane, i])))
                         for i in range(R)]
                wp = [zero_unless(f32(wv[i] - t[i]), i < nv) for i in range(R)]
                for i in range(max(0, min(nv, R))):
                    out[r + i] = wp[i]
                    written[r + i] += 1
                for wid in range(WV):
                    for q in range(slots):
                        c = wid + WV * q
                        if c < k:
                            v = vals[(wid, lane, q)]
                            acc[c] += sum(float(v[i] if i < nv else 0.0) * float(wp[i]) for i in range(R))
    assert np.all(written == 1)
    Vm = V[:k, :n]
    ref = w[:n].astype(np.float64) - (h[:k].astype(np.float64) @ Vm.astype(np.float64))
    assert np.all(np.isfinite(out[:n]))
    assert np.allclose(out[:n], ref, rtol=1e-5, atol=1e-5)
    assert np.all(np.isfinite(acc))
    assert np.allclose(acc[:k], Vm.astype(np.float64) @ out[:n].astype(np.float64), rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("n,k,slots,B,WV", [(1000, 5, 4, 3, 4), (700, 17, 8, 2, 4), (513, 40, 6, 2, 8),
                                            (300, 50, 8, 4, 8), (130, 3, 4, 5, 4), (1, 1, 4, 1, 4)])
def test_update_step_stand_in_rows(n, k, slots, B, WV):
    update_step_fp32(n, k, slots, B, WV)
