"""Comparison helpers shared by the GPU parity tests (no GPU code, no method arithmetic)."""
import numpy as np


def compare_traces(amr, gout, ores, what=""):
    """Per-ray segment lists of a GPU render against the oracle's: (leaf, patch, n, level, t_a,
    t_b) bit for bit.  Rays the oracle flags as edge cases (a ray along a leaf edge, where two
    slab planes may tie within one ulp) are excluded from the bit-exact check; their count is
    printed and must be zero, as it is for every pixel-centre ray of the views under test.
    Returns the number of rays compared."""
    g = amr.trace_records(gout)
    gn = gout["trace_n"].cpu().numpy()
    on = ores["trace_n"]
    flagged = int(np.count_nonzero(ores["flags"]))
    print("traces%s: %d rays, %d flagged as edge cases" % (" " + what if what else "", len(on), flagged))
    assert flagged == 0
    assert np.array_equal(gn, on)
    cap = g.shape[1]
    for q in range(len(on)):
        n = min(on[q], cap)
        a, b = g[q, :n], ores["trace"][q, :n]
        for f in ("leaf", "patch", "n", "level"):
            assert np.array_equal(a[f], b[f]), (q, f)
        assert np.array_equal(a["ta"], b["ta"]) and np.array_equal(a["tb"], b["tb"]), q
    return len(on)


def pixel_set(W, H, seed, nrandom=16384, crop=64, rows=4):
    """Seeded pixel sample of a W x H view: `nrandom` uniform random pixels, `rows` full rows
    spread over the height and a crop x crop block at the centre ([npix, 2] int32, (i, j))."""
    rng = np.random.default_rng(seed)
    pix = [np.stack([rng.integers(0, W, nrandom), rng.integers(0, H, nrandom)], 1)]
    for r in range(rows):
        row = min(H - 1, (H * (2 * r + 1)) // (2 * rows) + 3)
        pix.append(np.stack([np.arange(W), np.full(W, row)], 1))
    c = min(crop, W, H)
    cy, cx = (H - c) // 2, (W - c) // 2
    jj, ii = np.meshgrid(np.arange(cy, cy + c), np.arange(cx, cx + c), indexing="ij")
    pix.append(np.stack([ii.ravel(), jj.ravel()], 1))
    return np.ascontiguousarray(np.concatenate(pix), dtype=np.int32)
