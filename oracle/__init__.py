"""FP64 CPU oracle for the DPG local solve -- test infrastructure only.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import
this package.  It shares no code with the HIP path.

  dpg_oracle   forms (pointwise, and by App. A's real block matrices) and the
               local solve (LU; Jacobi-scaled Cholesky)
  xsolve       the local solve of given FP64 inputs in extended precision
  dpg_assembly condensation, trace numbering, assembly, CG, reconstruction
  dpg_power    power dissipation;  dpg_marking  Doerfler marking
"""
