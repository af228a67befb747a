"""FP64 CPU oracle for the DMTS-NC hot path -- TEST INFRASTRUCTURE ONLY.

This package is the slow, plain reference that the GPU path is checked
against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may import it; the product (``paper_2602_14975_amd``)
never does, and the two share no code.  Seeded inputs come from ``synth``,
which holds none of the method's arithmetic.

Everything is float64 on the CPU (numpy, or plain PyTorch CPU ops where a
gradient is needed; ``torch.autograd`` is used as a library routine to
differentiate the energy and the non-conservative force model).

Modules
-------
neighbors   minimum-image pair lists, brute force O(N^2) and a cell list
models      Bessel basis, cutoffs, the conservative message-passing energy and
            its forces, the distilled non-conservative force model (paper,
            Methods: "Model architecture") and its weight gradient
integrator  Philox-4x64-10 normals, BAOAB, BAOAB-RESPA / DMTS-NC (Algorithm
            1), hydrogen mass repartitioning, per-species friction
analysis    temperature, kinetic energy, O-O radial distribution, errors

Parity status: every function is pinned by tests under ``tests/`` marked
``not gpu``; the pins are listed in each module's docstring.  Agreement with
the paper's trained FeNNix-Bio1(M)/NC models is unpinned (no weights exist).
"""
