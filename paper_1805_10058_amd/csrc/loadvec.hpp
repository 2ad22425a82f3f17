// Load vector of the manufactured solutions (Sec. 6.2) and L2 error (internal header).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace cd {

// Device copy of one axis's quadrature tables (setup.hpp, QuadAxis).
struct QuadDev {
    const double* x;
    const double* w;
    const double* val;
    const double* der;
    const int* f0;
    int n, p, q, m, Q;
};

// b = load vector of the d-dimensional manufactured solution (component-major
// layout of the system); work: load_vector_work(d, ax) doubles.
void launch_load_vector(int d, const QuadDev* ax, double alpha, double beta, double* b, double* work, hipStream_t s);
size_t load_vector_work(int d, const QuadDev* ax);
// part[0 .. nparts) = partial sums of the squared L2 error of the
// coefficient vector x against the manufactured solution; work:
// l2_error_work(d, ax) doubles.
void launch_l2_error(int d, const QuadDev* ax, const double* x, double* work, double* part, int nparts, hipStream_t s);
size_t l2_error_work(int d, const QuadDev* ax);

}  // namespace cd
