"""FP64 CPU oracle for the slimLS hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct numpy/scipy code written from the paper
(Chung, Chung, Slagel, Tenorio, "Sampled limited memory methods for massive
linear inverse problems", arXiv 1912.07962).  Only ``tests/``, the smoke
check in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may use
it; the GPU library never imports, links or calls it, and it shares no code
with the GPU path (only the seeded generators in ``synth`` feed both).

Modules
  geometry  -- scan geometry and the closed-form Joseph weight (sec. 4.3 setup)
  system    -- explicit CSR rows of A for blocks of angles; dense brute force
  slimls    -- the slimLS iteration, eq. (ram) with B_k of eq. (B_k), C_k = I,
               alpha = 1/lambda; dual (Gram) form, Woodbury form, primal form
  sampler   -- counter-based SplitMix64 + Fisher-Yates random-cyclic schedule

Parity status per function is listed in each module header.
"""
from . import geometry, system, slimls, sampler  # noqa: F401
