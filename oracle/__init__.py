"""FP64 CPU oracle for the IgA curl-div solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: it exists so that ``tests/``, the smoke
check and the CPU-baseline leg of the benchmark can compare the GPU library
against a plain, slow, obviously correct implementation written from the
paper (Mazza, Manni, Ratnani, Serra-Capizzano, Speleers, "Isogeometric
analysis for 2D and 3D curl-div problems: spectral symbols and fast iterative
solvers").  It shares no code with the GPU library.

Modules
-------
bspline   : knots, Cox-de Boor recursion, cardinal B-splines       (Sec. 3.1)
matrices  : 1D mass / advection / stiffness matrices, Toeplitz T    (Sec. 3.2, 6.1)
assembly  : literal 2x2 / 3x3 block matrices, Kronecker apply       (Sec. 4.1, 4.2)
symbols   : spectral symbols m_p, a_p, s_p, f^{p,alpha,beta}, g_p   (Sec. 3.2, 5)
transfer  : paper prolongator and knot-insertion prolongator        (Sec. 6.1)
solvers   : direct solve, plain CG, fast diagonalization            (Sec. 6, Remark 6.1)
mim       : the paper's multi-iterative method with exact Gauss-Seidel (Sec. 6.1-6.2)
method    : the parallel-smoother V-cycle and flexible CG that the GPU library
            computes, written out step by step (Sec. 6.1 with the readings
            listed in its module docstring)
loadvec   : manufactured-solution load vectors of the numerical examples (Sec. 6.2)
"""
