"""Hybro placer hot path on one AMD Instinct MI355X (gfx950).

Modules:
  * hybro     -- ctypes binding of libhybro.so (the C ABI in include/hybro.h) and the Placer
                 convenience class; fails loudly when the library is missing.
  * build     -- compiles the HIP sources in csrc/ into libhybro.so in-tree.
  * netgen    -- seeded synthetic netlists (tiny / mid / large / mid_mm, fillers).
  * alg1      -- Hybro's outer loop (Alg. 1) on the device: place, perturb, keep the best.
  * autotune  -- timing tuner for the charge scatter's grouping policy.
  * serve     -- a serving loop for mixed placement jobs sharing one GPU.
  * autograd  -- torch.autograd wrappers around the evaluation.
"""
