"""LDS layouts of the line FFTs and the FP64 overlap tiles against a bank model.

The kernels space the x-line exchange buffers by a table of strides
(``x_line_stride`` in ``csrc/fft_line.h``) and store the FP64 overlap's rows
through a column permutation (``kperm`` in ``csrc/mfma_f64.h``).  These tests
re-derive both from a model of the LDS banks: 4-byte banks, an access of
``W``-word values processed in groups of ``banks / W`` lanes, each group
taking as many cycles as the most words any bank holds.  With 32 banks it
reproduces the measured bank-conflict counters of the previous layouts (the
x pass of h psi at twice its conflict-free cycles; the FP64 recombination's
transposing stores at four times).
"""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1610_07522_amd", "csrc")

FACT = {}
for n, r1, r2 in re.findall(r"struct Fact<(\d+)>\s*\{\s*static constexpr int R1 = (\d+), R2 = (\d+);",
                            open(os.path.join(CSRC, "sky_common.h")).read()):
    FACT[int(n)] = (int(r1), int(r2))


def excess(accesses, banks, words):
    """Cycles above the conflict-free count over a list of 64-lane accesses
    (value indices; None for an inactive lane)."""
    group = banks // words
    extra = 0
    for acc in accesses:
        for g0 in range(0, 64, group):
            lanes = [a for a in acc[g0:g0 + group] if a is not None]
            if not lanes:
                continue
            per_bank = {}
            for a in set(lanes):
                for w in range(words * a, words * a + words):
                    per_bank.setdefault(w % banks, set()).add(w)
            extra += max(len(v) for v in per_bank.values()) - 1
    return extra


def line_exchange(n, spins, stride, along_x):
    """Every LDS access of the two-stage exchange of one wave's lines."""
    r1, r2 = FACT[n]
    rt = max(r1, r2)
    lpw = 64 if rt == 4 else 32
    lanes = []
    for t in range(64):
        if along_x:
            j, line = t % rt, t // rt
        else:
            j, line = t // lpw, t % lpw
        lanes.append((line, j))
    row = r2 + 1
    out = []
    for s in range(spins):
        for k1 in range(r1):
            out.append([l * stride + (s * r1 + k1) * row + j if j < r2 else None for l, j in lanes])
        for k2 in range(r2):
            out.append([l * stride + (s * r1 + j) * row + k2 if j < r1 else None for l, j in lanes])
    return out


def header_strides():
    text = open(os.path.join(CSRC, "fft_line.h")).read()
    one = [int(v) for v in re.search(r"one\[6\] = \{([^}]*)\}", text).group(1).split(",")]
    two = [int(v) for v in re.search(r"two\[6\] = \{([^}]*)\}", text).group(1).split(",")]
    sizes = [8, 16, 24, 32, 48, 64]
    return {(n, 1): one[i] for i, n in enumerate(sizes)} | {(n, 2): two[i] for i, n in enumerate(sizes)}


def test_x_line_strides_are_the_least_conflicting():
    for (n, spins), stride in header_strides().items():
        r1, r2 = FACT[n]
        low = spins * r1 * (r2 + 1)
        assert stride >= low, (n, spins)

        def cost(v):
            return sum(excess(line_exchange(n, spins, v, True), b, w) for b in (32, 64) for w in (2, 4))

        best = min(cost(v) for v in range(low, low + 64))
        assert cost(stride) == best, (n, spins, stride)
        if n != 24:   # lines of 24 points straddle waves; elsewhere no bank is shared
            assert best == 0, (n, spins)


def test_odd_stride_serves_y_and_z_and_fails_x():
    for n in FACT:
        for spins in (1, 2):
            r1, r2 = FACT[n]
            odd = spins * r1 * (r2 + 1) + 1
            for b in (32, 64):
                for w in (2, 4):
                    assert excess(line_exchange(n, spins, odd, False), b, w) == 0, (n, spins, b, w)
    # the measured case: x pass at 48^3, complex64, two spin components, 32 banks
    acc = line_exchange(48, 2, 109, True)
    assert excess(acc, 32, 2) > 0
    assert excess(line_exchange(48, 2, header_strides()[(48, 2)], True), 32, 2) == 0


def kperm(kk):
    src = open(os.path.join(CSRC, "mfma_f64.h")).read()
    assert "return (kk >> 1) | ((kk & 1) << 3);" in src
    return (kk >> 1) | ((kk & 1) << 3)


def test_fp64_overlap_permutation():
    kp, kc = 17, 16
    assert sorted(kperm(k) for k in range(kc)) == list(range(kc))
    # loader: thread -> (row tid/4, contraction 4 (tid%4) + e), one store per e
    stores = [[(t >> 2) * kp + kperm((t & 3) * 4 + e) for t in range(64 * w, 64 * w + 64)]
              for w in range(4) for e in range(4)]
    plain = [[(t >> 2) * kp + (t & 3) * 4 + e for t in range(64 * w, 64 * w + 64)]
             for w in range(4) for e in range(4)]
    # MFMA operand reads: lane -> (row lane%16, contraction kk + lane/16)
    reads = [[(wm * 32 + i * 16 + (l & 15)) * kp + kperm(kk + (l >> 4)) for l in range(64)]
             for wm in range(2) for i in range(2) for kk in range(0, kc, 4)]
    assert excess(plain, 32, 4) > 0
    assert excess(stores, 32, 4) == 0
    assert excess(reads, 32, 4) == 0


def test_fp64_recombination_loader():
    kp = 17
    # thread -> (contraction tid/16, columns tid%16 + 16 e), stored transposed
    new = [[((t & 15) + 16 * e) * kp + (t >> 4) for t in range(64 * w, 64 * w + 64)]
           for w in range(4) for e in range(4)]
    old = [[((t & 15) * 4 + e) * kp + (t >> 4) for t in range(64 * w, 64 * w + 64)]
           for w in range(4) for e in range(4)]
    assert excess(old, 32, 4) > 0
    assert excess(new, 32, 4) == 0
    src = open(os.path.join(CSRC, "k_gemm.hip")).read()
    assert "const int col = lc + 16 * e, b = b0 + col;" in src
