// Host LAPACK/BLAS (FP64 complex) resolved at run time from Intel MKL's
// single dynamic library. Only the handful of routines the FP64 setup needs.
#pragma once
#include <complex>
#include <string>

namespace scw {

using zc = std::complex<double>;

struct Lapack {
  void (*zgeev)(const char*, const char*, const int*, zc*, const int*, zc*, zc*,
                const int*, zc*, const int*, zc*, const int*, double*, int*) = nullptr;
  void (*zgetrf)(const int*, const int*, zc*, const int*, int*, int*) = nullptr;
  void (*zgetrs)(const char*, const int*, const int*, const zc*, const int*,
                 const int*, zc*, const int*, int*) = nullptr;
  void (*zgemm)(const char*, const char*, const int*, const int*, const int*,
                const zc*, const zc*, const int*, const zc*, const int*,
                const zc*, zc*, const int*) = nullptr;
  void (*zgecon)(const char*, const int*, const zc*, const int*, const double*,
                 double*, zc*, double*, int*) = nullptr;
  double (*zlange)(const char*, const int*, const int*, const zc*, const int*,
                   double*) = nullptr;
  int (*set_threads_local)(int) = nullptr;    // per calling thread
  void (*set_threads)(int) = nullptr;         // process default
  bool ok = false;
  std::string error;
};

// Loads once per process; later calls return the same table.
const Lapack& lapack();

}  // namespace scw
