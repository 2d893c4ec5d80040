"""phi-function actions of Kronecker-sum matrices on AMD MI355X (gfx950).

    from paper_2211_00696_amd import phiq
    with phiq.Handle(0) as h:
        out, report = h.action([Ax, Ay, Az], t, p, v, tol=1e-8)

``phiq`` binds the C-ABI library libphiq.so (include/phiq.h); the HIP
kernels do all the work.  ``inputs`` builds seeded synthetic workloads.
"""
__all__ = ["phiq", "inputs", "build"]
