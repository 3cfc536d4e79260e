"""CPU restatement of the pipelined update + projection sweep of a bf16 basis
(no GPU): the block's row range, the two register sets filled one step ahead,
the stand-in row for lanes past the range and columns past k, the steps run
in pairs (an odd count gets one masked step), and the masking of w'.

Checks, for ragged and empty row ranges and every column class, that every
load stays inside the basis (m + 1 columns of ldv rows) and the work vector
(ldv rows), that every row of the block's range is updated exactly once, and
-- with NaN in the padded rows past n, which the library never writes -- that
w' and the partial projections come out finite and equal (w', bitwise in the
kernel's summation order) or close (the projections) to a direct evaluation."""
import numpy as np
import pytest

WAVE, R = 64, 4
STEP = WAVE * R


def block_rows(n, B, b):
    chunk = -(-n // B)
    chunk = (chunk + 63) & ~63
    a = b * chunk
    return min(a, n), min(a + chunk, n)


def wave_sum(p):
    # the parts of the block's waves added in the kernel's fixed order
    t = np.float32(np.float32(p[0] + p[1]) + np.float32(p[2] + p[3]))
    if len(p) == 8:
        t = np.float32(t + np.float32(np.float32(p[4] + p[5]) + np.float32(p[6] + p[7])))
    return t


def sweep(n, k, slots, B, WV=4, m=None, seed=0):
    f32 = np.float32
    m = m if m is not None else k
    ldv = -(-n // 128) * 128
    rng = np.random.default_rng(seed)
    V = np.full((m + 1) * ldv, np.nan, f32)
    for c in range(m + 1):
        V[c * ldv:c * ldv + n] = rng.uniform(-1, 1, n)
    w = np.full(ldv, np.nan, f32)
    w[:n] = rng.uniform(-1, 1, n)
    h = np.zeros(WV * slots, f32)
    h[:k] = rng.uniform(-1, 1, k)
    w_out = np.full(ldv, np.nan, f32)
    written = np.zeros(n, int)
    acc_total = np.zeros(WV * slots, np.float64)
    for b in range(B):
        r0, r1 = block_rows(n, B, b)
        rz = r0 & ~63

        def load_step(base):
            vals = {}
            for wid in range(WV):
                for lane in range(WAVE):
                    r = base + R * lane
                    for q in range(slots):
                        c = wid + WV * q
                        ok = c < k and r1 - r > 0
                        a = c * ldv + r if ok else rz
                        assert 0 <= a and a + R <= (m + 1) * ldv, (b, base, wid, lane, q)
                        vals[(wid, lane, q)] = V[a:a + R].copy()
            return vals

        npairs = -(-(r1 - r0) // (2 * STEP))
        cur = load_step(r0)
        for st in range(2 * npairs):
            base = r0 + st * STEP
            nxt = load_step(base + STEP)
            # per wave partial sums of V h over its columns, then the waves in order
            part = np.zeros((WV, WAVE, R), f32)
            for wid in range(WV):
                for lane in range(WAVE):
                    r = base + R * lane
                    nv = r1 - r
                    s = np.zeros(R, f32)
                    for q in range(slots):
                        v = cur[(wid, lane, q)]
                        for i in range(R):
                            s[i] = f32(s[i] + f32(h[wid + WV * q] * (v[i] if i < nv else f32(0))))
                    part[wid, lane] = s
            for lane in range(WAVE):
                r = base + R * lane
                nv = r1 - r
                wa = r if nv > 0 else rz
                assert 0 <= wa and wa + R <= ldv
                wv = w[wa:wa + R].copy()
                t = np.array([wave_sum(part[:, lane, i]) for i in range(R)], f32)
                wp = np.where(np.arange(R) < nv, f32(wv - t), f32(0))
                for i in range(min(max(nv, 0), R)):
                    w_out[r + i] = wp[i]
                    written[r + i] += 1
                for wid in range(WV):
                    for q in range(slots):
                        c = wid + WV * q
                        if c < k:
                            v = cur[(wid, lane, q)]
                            acc_total[c] += sum(float(v[i] if i < nv else 0.0) * float(wp[i]) for i in range(R))
            cur = nxt
    assert np.all(written == 1)
    Vm = V[:k * ldv].reshape(k, ldv)[:, :n]
    # w' in the kernel's order: per wave over its columns, then the waves in order
    ref = np.empty(n, f32)
    for r in range(n):
        s = [f32(0)] * WV
        for wid in range(WV):
            for q in range(slots):
                c = wid + WV * q
                s[wid] = f32(s[wid] + f32(h[c] * (Vm[c, r] if c < k else f32(0))))
        ref[r] = f32(w[r] - wave_sum(s))
    assert np.array_equal(w_out[:n], ref)
    assert np.all(np.isfinite(acc_total))
    assert np.allclose(acc_total[:k], Vm.astype(np.float64) @ ref.astype(np.float64), rtol=1e-6, atol=1e-9)


@pytest.mark.parametrize("n,k,slots,B,WV", [(1000, 5, 4, 3, 4), (1000, 16, 4, 2, 4), (700, 17, 8, 2, 4),
                                            (513, 40, 12, 1, 4), (300, 50, 16, 4, 4), (64, 3, 4, 2, 4), (1, 1, 4, 1, 4),
                                            (900, 101, 16, 2, 8), (257, 70, 12, 3, 8)])
def test_pipelined_sweep_bounds_and_values(n, k, slots, B, WV):
    sweep(n, k, slots, B, WV)


def test_empty_block_ranges():
    # more blocks than 64-row chunks: the trailing blocks get r0 = r1 = n and
    # make only their first (stand-in) basis load
    sweep(130, 6, 4, 5)
