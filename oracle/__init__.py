"""Oracle for the w-gridding measurement operator (arXiv:2010.10122).

TEST INFRASTRUCTURE ONLY.  Only tests/, the ``smoke()`` check in
__graft_entry__.py and the ``cpu_baseline`` leg of bench.py may import, call,
link or execute anything in this directory.  The product package never does,
and no code is shared between the two: the oracle is a plain, slow, obviously
correct CPU FP64 implementation written from the paper.

Modules
-------
kernel  -- modified ES kernel (eq. semicircle2), its Fourier transform psi,
           map error function (eq. maperror), Appendix-A parameter tables.
plan    -- grid size, w-plane geometry (Sect. 2) and the binning spec (Sect. 4.3).
o1      -- O1: direct DFT of eq. (3) and its adjoint (C, OpenMP; dft.c).
o2      -- O2: plain w-gridding (de)gridder following eqs. (R1)-(R3), (Rad1)-(Rad2).
"""
