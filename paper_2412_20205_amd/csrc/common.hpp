// Shared definitions of the HIP library (host and device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

namespace igamg {

// Failure raised inside the library and turned into an igamg_status at the ABI.
struct Error : std::runtime_error {
    int status;
    Error(int s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define IGAMG_HIP(call)                                                                 \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            throw ::igamg::Error(-3, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr int kBlock = 256;       // threads per block of the streaming kernels
constexpr int kMaxMu = 4;         // largest cycle index of Algorithm 2 accepted
constexpr int kNumXcd = 8;        // accelerator complex dies of an MI355X
constexpr int kQrRows = 512;      // rows of one tall-skinny QR panel (LDS <= 37 KB)
constexpr int kMaxQ = 8;          // largest restart number q
constexpr int kMaxCols = kMaxQ + 1;

constexpr int kMaxKrylov = 30;    // largest restart length of flexible GMRES

// Basis vectors passed by value to the Krylov kernels.
struct VecPtrs {
    const double* v[kMaxKrylov + 1];
};

// Iterate pointers s_0 .. s_{q+1} passed by value to the extrapolation kernels.
struct IterPtrs {
    const double* s[kMaxQ + 2];
};

// Device-side result of the small extrapolation solve.
struct ExtrapCoeffs {
    double gamma[kMaxCols];
    double alpha[kMaxCols];
    int info;  // 0 regular, 1 lucky breakdown, -1 lambda ~ 0, -2 non-finite
    int lucky_col;
    double gres;  // ||sum_j gamma_j Delta s_j|| = ||R gamma|| (generalised residual; NaN on breakdown)
    double d0;    // ||Delta s_0|| = |R_00|
};

}  // namespace igamg
