"""FP64 CPU oracle for the multi-scale S-fraction reduced-order model.

TEST INFRASTRUCTURE ONLY. Nothing in the product package imports, calls,
links or executes anything here; only the test suite, the smoke check and
the benchmark's CPU-baseline leg may use it. It shares no code with the HIP
path: the two meet only through the seeded generators in ``synth``.

Each function is a plain, slow, obviously-correct restatement of the paper
(Druskin, Mamonov, Zaslavsky, "Multi-scale S-fraction reduced-order models
for massive wavefield simulations"), citing the section or equation it
follows:

* ``fine``      - fine-grid pencil (Sec. 1, eq. wave_fll), leapfrog, and the
                  exact modal solution of the leapfrog recurrence;
* ``partition`` - Cartesian coarse cells, skeleton pieces, voxel-wise
                  operator splitting (Sec. 2, eq. splitN_c), boundary bases
                  (Sec. 4.1);
* ``rom_cell``  - per-cell rational block Krylov projection (Sec. 4.2,
                  eqs. npks, tfprj), block Lanczos (App. C, eq. NtDtri) and
                  the S-fraction change of variables (App. C, eq. GammaTrans);
* ``rom_global``- boundary conjugation and the global time-domain ROM
                  (Sec. 6, eqs. intrtstep_td, bdrytstep) with leapfrog.

Readings of places where the paper is ambiguous or misprinted are stated
in the docstrings where they are used.
"""
