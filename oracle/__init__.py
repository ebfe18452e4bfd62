"""CPU FP64 oracle for the two-level Schwarz / Bezier coarse-space GMRES path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything in this
package.  The product library (``paper_2408_03571_amd``) never imports it and
shares no code with it; the only common module is ``workloads`` (seeded input
generators, no method arithmetic).

Plain, slow, obviously-correct NumPy/SciPy in complex128 (complex64 only where
the mixed-precision form rounds the local solves on purpose).  Each function
cites the passage of arXiv 2408.03571 it follows:

* ``problem``  Sec. 2, model problems MP-1 / MP-2 and eq. (LS_final)
* ``decomp``   Sec. 3, the overlapping decomposition and R_i, D_i
* ``bezier``   Sec. 4, eq. (GCS:HO_R_0), the Bezier restriction R_0
* ``bandlu``   Sec. 3, exact local / coarse solves (hand-written band LU)
* ``schwarz``  Sec. 3, eqs. (DDM:SO_AS) and (DDM:SO_SAS)
* ``gmres``    Sec. 5, GMRES with a relative tolerance
* ``eigen``    Sec. 2, MP-1 (closed-form discrete solution used as a pin)
* ``adjoint``  gradient of a receiver misfit with respect to k^2

Parity unpinned: there is no absolute reference for MP-2 solution values at
n >= 257 (no closed form, and the paper prints no solution values); there the
oracle is trusted through the small-grid pins and its own true residual.
The paper's printed iteration counts (Tables 1-4) are a soft check only.
"""
