// C wrapper of the library's host Jacobi eigensolver, compiled into a CPU-only
// test library together with paper_2502_00152_amd/csrc/dense_eig.cpp.
#include <complex>
namespace hisq {
int heev_jacobi(int n, std::complex<double> *A, double *w, std::complex<double> *Z, int max_sweeps);
}
extern "C" int test_heev(int n, double *A, double *w, double *Z, int max_sweeps) {
    return hisq::heev_jacobi(n, reinterpret_cast<std::complex<double> *>(A), w,
                             reinterpret_cast<std::complex<double> *>(Z), max_sweeps);
}

namespace hisq {
int syev_qr(int n, double *A, double *w, double *Z);
}
extern "C" int test_syev(int n, double *A, double *w, double *Z) {
    return hisq::syev_qr(n, A, w, Z);
}

namespace hisq {
int heev_qr(int n, std::complex<double> *A, double *w, std::complex<double> *Z);
}
extern "C" int test_heev_qr(int n, double *A, double *w, double *Z) {
    return hisq::heev_qr(n, reinterpret_cast<std::complex<double> *>(A), w,
                         reinterpret_cast<std::complex<double> *>(Z));
}
