// Launchers of the polynomial chaos kernels (gpc_kernels.hip).
#pragma once

#include "edf_internal.h"

namespace edf {

constexpr int kGpcMaxM = 4;       // parameters of the expansion
constexpr int kGpcMaxDeg = 8;     // largest degree of one parameter
constexpr int kGpcMaxCoef = 128;  // expansion terms

// W[q][i] = w_i Psi_q(theta_i) / Q_q; theta [S][ldt], idx [nc][M], Q [nc]
void launch_gpc_weights(int S, int M, int nc, const double* theta, int ldt, const double* w,
                        const int* idx, const double* Q, double* W, hipStream_t st);
// C[q][v] = sum_i W[q][i] F[i][v]; F [S][Nc], C [nc][Nc]
void launch_gpc_project(int S, int Nc, int nc, const double* W, const double* F, double* C,
                        hipStream_t st, hipEvent_t ev0, hipEvent_t ev1);
// mean = C[0], var = sum_{q >= 1} Q_q C[q]^2
void launch_gpc_moments(int Nc, int nc, const double* C, const double* Q, double* mean,
                        double* var, hipStream_t st);
// B[q][s] = Psi_q(theta_s) for a batch of n points (theta [n][M]); rows q in [nc, ncp)
// and columns s in [n, ldb) are zero; B [ncp][ldb]
void launch_gpc_basis(int n, int ldb, int nc, int ncp, int M, const int* idx, const double* theta,
                      double* B, hipStream_t st);
// partial[chunk0 + y][v] = #{s in chunk y of the batch : sum_q C[q][v] B[q][s] > thr} for
// the batch's n points; chunk is a multiple of 64 and n <= ldb, ldb a multiple of 64
void launch_gpc_exceed(int Nc, int nc, const double* C, const double* B, int ldb, int n, int chunk,
                       int chunk0, int n_chunks, double thr, int* partial, hipStream_t st,
                       hipEvent_t ev0, hipEvent_t ev1);
// prob[v] = sum_y partial[y][v] / Ns
void launch_gpc_count(int Nc, int n_chunks, int Ns, const int* partial, double* prob,
                      hipStream_t st);

}  // namespace edf
