// Rosenbrock method Rodas4 (Hairer & Wanner, Solving ODEs II, sec. IV.7) in
// the transformed variables u_i = sum_j gamma_ij k_j:
//   (I/(gamma h) - J) u_i = f(y0 + sum_j a_ij u_j) + sum_j (c_ij / h) u_j,
// six stages; stiffly accurate, so the sixth stage argument is the embedded
// solution, y1 = that argument + u_6, and u_6 estimates the local error.
// Coefficients as published with the method (16 significant digits).
// Step-size control: scaled RMS error norm, h_new = h min(5, max(0.2,
// 0.9 err^(-1/4))), no growth right after a rejection, last step clipped to
// the interval end.
#pragma once
#include <hip/hip_runtime.h>

namespace adm1 {

constexpr double kR4Gamma = 0.25;
constexpr int kR4Stages = 6;

__device__ constexpr double kR4A[6][5] = {
    {0.0, 0.0, 0.0, 0.0, 0.0},
    {1.544, 0.0, 0.0, 0.0, 0.0},
    {0.9466785280815826, 0.2557011698983284, 0.0, 0.0, 0.0},
    {3.314825187068521, 2.896124015972201, 0.9986419139977817, 0.0, 0.0},
    {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950, 0.0},
    {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950, 1.0},
};
__device__ constexpr double kR4C[6][5] = {
    {0.0, 0.0, 0.0, 0.0, 0.0},
    {-5.6688, 0.0, 0.0, 0.0, 0.0},
    {-2.430093356833875, -0.2063599157091915, 0.0, 0.0, 0.0},
    {-0.1073529058151375, -9.594562251023355, -20.47028614809616, 0.0, 0.0},
    {7.496443313967647, -10.24680431464352, -33.99990352819905, 11.70890893206160, 0.0},
    {8.083246795921522, -7.981132988064893, -31.52159432874371, 16.31930543123136,
     -6.058818238834054},
};

// Step-size factor of the controller from the scaled error (NaN/inf: 0.2).
__device__ __forceinline__ double step_factor(double err)
{
    if (!(err < INFINITY)) return 0.2;
    if (err == 0.0) return 5.0;
    return fmin(5.0, fmax(0.2, 0.9 / sqrt(sqrt(err))));
}

}  // namespace adm1
