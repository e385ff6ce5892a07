"""FP64 CPU oracle for the split-step turbulence path (TurPy, arXiv 2604.07248).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct
restatement of what the GPU path computes, written from the paper: phase-screen
synthesis from the modified von Karman PSD (App. B Eq. S16, App. C Eq. S17-S18),
Lane subharmonics (Sec. 2.2 Eq. 2-3), the split-step step (Sec. 2.1 Eq. 1), the
frozen-flow / AR(1) screen evolution (Sec. 2.3 Eq. 4-5), ensemble statistics
(Sec. 3.3, Eq. S25) and the dual-domain receiver (Sec. 2.5 / Sec. 4).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with the HIP library and imports
nothing from it; both sides are fed by the seeded input generators in
``paper_2604_07248_amd.workloads``.  Library primitives used as single steps:
``numpy.fft`` (pocketfft) for the DFTs, numpy elementwise math in float64.
"""

from . import philox, noise, screens, propagate, evolve, stats, receiver  # noqa: F401
