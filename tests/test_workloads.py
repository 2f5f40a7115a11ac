"""The seeded generators: the time-lapse survey's structure (CPU only)."""
import numpy as np

import workloads as W


def test_timelapse_survey_structure():
    wl = W.timelapse_survey(nx=120, nz=80, h=10.0, T=300.0, nvint=5, nsrc=8, nrec=50, shots_per_vintage=3,
                            nbl=12, iteration=2)
    assert wl.nwindow == 5 and wl.nshot == 15
    assert [s.window for s in wl.shots] == [i for i in range(5) for _ in range(3)]
    # the plume only lowers the wavespeed, by at most the drop, and grows with the vintage
    base = wl.v[0] / (1.0 - 0.05 * W.plume_mask(wl.v[0].shape, wl.h, 1, 5))
    sizes = []
    for i in range(5):
        ratio = wl.v[i] / base
        assert ratio.max() <= 1.0 + 1e-12 and ratio.min() >= 0.95 - 1e-12
        sizes.append(int((ratio < 1.0 - 1e-9).sum()))
    assert all(a <= b for a, b in zip(sizes, sizes[1:])) and sizes[-1] > sizes[0] > 0
    # crosswell geometry inside the physical model: sources in the left well, receivers right
    L = (np.array(wl.v[0].shape[::-1]) - 1) * wl.h
    for s in wl.shots:
        assert s.src[0] < 0.2 * L[0] and 0 <= s.src[2] <= L[1]
        assert np.all(s.rec[:, 0] > 0.8 * L[0]) and np.all((s.rec[:, 2] >= 0) & (s.rec[:, 2] <= L[1]))
    # sampling with replacement is reproducible per iteration and differs between iterations
    again = W.timelapse_survey(nx=120, nz=80, h=10.0, T=300.0, nvint=5, nsrc=8, nrec=50, shots_per_vintage=3,
                               nbl=12, iteration=2)
    other = W.timelapse_survey(nx=120, nz=80, h=10.0, T=300.0, nvint=5, nsrc=8, nrec=50, shots_per_vintage=3,
                               nbl=12, iteration=3)
    z = lambda w: [float(s.src[2]) for s in w.shots]
    assert z(again) == z(wl) and z(other) != z(wl)
