"""MI355X-native hp space-time multigrid for the instationary Stokes equations
(Q_{r+1}/P_r^disc x DG(k) slabs, cell Vanka smoother, FGMRES).

The compute path is the HIP library ``libstmg.so`` (built in-tree by
``paper_2502_09159_amd.build``); ``paper_2502_09159_amd.stmg`` is its thin
ctypes binding.  Importing the binding raises if the library is missing.
"""
