"""CPU FP64 oracle of the immersed-boundary projection step (Ong & Miura).

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, independent CPU
implementation of what the projection step computes, written from the paper.
Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import it; the product path (the HIP library and its binding) never does,
and it shares no code with that path. Inputs come from the seeded generators
in ``paper_1807_10504_amd.workloads`` (data only).

Modules and the parts of the paper they follow:
  kernel     -- cosine kernel phi (eq cherby), its integral H (eq new_hea) and
                the region values (eq new_hea2)
  transfer   -- velocity interpolation (eq jump_condu) and conventional
                delta-function spreading (eq delta_vec)
  heaviside  -- discrete Heaviside from offset polygons / polyhedra
                (Section 3.2, eqs new_hea, new_hea2)
  force      -- face surface tension f and the irrotational delta vector
                (eq delta_hea_xy)
  poisson    -- density from the indicator (eq indicator), the projection
                Poisson problem (eqs ps, ns2_new) and its multigrid solution
  bspline    -- least-squares B-spline relocation and curvature (Section 4)
  surface3d  -- sphere-mesh curvature force (builder's 3D extension)
  step       -- one projection step composed from the above
  diag       -- pressure jump, kinetic energy, force ratio, discrete curl

Every function is FP64 NumPy or plain Python unless stated otherwise.
"""
