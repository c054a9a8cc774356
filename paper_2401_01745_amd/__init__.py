"""MI355X emRKC: explicit exponential multirate Runge-Kutta-Chebyshev time
stepping of the monodomain model on one GPU.

The computation lives in the HIP library ``libemrkc.so`` (C ABI declared in
``include/emrkc.h``); this package only marshals arguments to it
(``paper_2401_01745_amd.emrkc``) and holds the build script.
"""
__all__ = ["emrkc", "build"]
