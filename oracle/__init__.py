"""FP64 CPU oracle for the NASGabor and degree-3 SH appearance path.

TEST INFRASTRUCTURE ONLY. This package is the slow, plain, obviously-correct
reference that the HIP kernels are checked against. Only ``tests/``, the
smoke check in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py``
may import it. The product path (``paper_2606_09794_amd``) never imports,
calls or links anything here, and this package imports nothing from the
product path: the two share no code, constants or helpers. Inputs come from
``workloads`` (random draws only).

Modules
-------
nasg_ref  NASGabor value, both normalisers, analytic gradients (paper
          Section 5.1, Supplementary Materials E and F) and the quaternion /
          view-direction chain rules.
sh3_ref   Real degree-3 spherical harmonics, value and gradient (Section 3.2).
nasg_paper  The paper's own lobe parametrisation (Supplementary C).
families  The other lobe families of the distribution table (Supplementary A).
raster_ref  Compositing into an image (Section 3.1) with colour, opacity and
          geometry gradients.
lr_ref    Training-rate scales and schedule.
metrics   Error metric used by the parity tests (scale-normalised error).
"""
