"""Host check of the tiling behind the one-tile super-resolution x-step.

The x-step of the 9-tap, factor-2 operator with mirrored boundary (Section
4.1) is taken per tile of the high-resolution grid: a block forms the
low-resolution residual r = A x - y on a window of samples [Ilo, Ihi] in LDS
and reads the adjoint at its pixels from there.  That is correct only if every
sample whose blur footprint reaches a pixel of the tile (directly or through a
mirrored copy) lies in the window.  The window formulas are restated here and
checked, axis by axis, against the samples found by brute force from the
operator's definition, for every image size up to 200 and the tile sizes the
kernels use; also that the window fits the LDS arrays sized for it, that the
interior fast path's clamped indices stay inside, and that the staged rows of
x need one reflection at most.
"""
import pytest

BS, F = 9, 2
R = (BS - 1) // 2
NS = (BS + F - 1) // F


def mirror(k, n):
    """Source index of padded position k under the mirrored (half-sample) extension."""
    while k < 0 or k >= n:
        k = -k - 1 if k < 0 else 2 * n - 1 - k
    return k


def samples_reading(n):
    """For each pixel, the set of samples I whose blur footprint (padded
    positions F I + a - R, a < BS) maps onto it: the definition of A, read
    backwards."""
    m = (n + F - 1) // F
    reads = [set() for _ in range(n)]
    for I in range(m):
        for a in range(BS):
            reads[mirror(F * I + a - R, n)].add(I)
    return m, reads


def window(i0, th, n, m):
    """The kernel's window of a tile starting at i0 (rows i0 .. i0 + th - 1)."""
    imax = min(i0 + th, n) - 1
    ilo = max(0, (i0 + R) // F - (NS - 1))
    ihi = min(m - 1, (imax + R) // F)
    return ilo, ihi


@pytest.mark.parametrize("th", [8, 16, 64])
def test_window_covers_every_sample_the_tile_reads(th):
    ni_max = (th - 1 + F - 1) // F + NS  # the LDS arrays' sample count per side
    for n in list(range(R + 1, 201)) + [511, 512, 513, 1024]:
        m, reads = samples_reading(n)
        for i0 in range(0, n, th):
            ilo, ihi = window(i0, th, n, m)
            assert 1 <= ihi - ilo + 1 <= ni_max, (n, th, i0)
            for i in range(i0, min(i0 + th, n)):
                assert reads[i], (n, i)
                assert min(reads[i]) >= ilo and max(reads[i]) <= ihi, (n, th, i0, i, sorted(reads[i]))
                # interior fast path: samples (i + R) / F - t, clamped at 0
                if R <= i < n - R:
                    for t in range(NS):
                        assert ilo <= max((i + R) // F - t, 0) <= ihi, (n, th, i, t)
            # staged rows of x: padded positions F Ilo - R .. F Ihi + R need one
            # reflection at most (the kernel's src_index does one)
            for k in (F * ilo - R, F * ihi + R):
                once = -k - 1 if k < 0 else (2 * n - 1 - k if k >= n else k)
                assert 0 <= once < n, (n, th, i0, k)


def test_window_matches_brute_force_exactly_in_the_interior():
    """Away from the edges the window is exactly the samples the tile reads
    (nothing staged in vain beyond the NS - 1 samples below the first pixel's)."""
    n, th = 512, 8
    m, reads = samples_reading(n)
    for i0 in range(2 * th, n - 2 * th, th):
        ilo, ihi = window(i0, th, n, m)
        need = set().union(*(reads[i] for i in range(i0, i0 + th)))
        assert ihi == max(need)
        assert ilo == min(need)
