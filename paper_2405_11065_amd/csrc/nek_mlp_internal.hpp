// Internal view of the initial-guess network shared by nek_mlp.hip and
// nek_x0.hip.  Internal header.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "nek_internal.hpp"
#include "nek_mlp.h"

// Parameters are FP32 masters P (dense, in the order of include/nek_mlp.h)
// with gradient G and Adam moments M, V; W*b are bfloat16 copies of the
// weights with row pitches ldin / ldh.  Activation buffers hold cap rows.
struct nek_mlp {
    int nin = 0, nh = 0, nout = 0, ldin = 0, ldh = 0, ldout = 0;
    hipStream_t stream = nullptr;
    long np = 0;
    long oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0;
    float *P = nullptr, *G = nullptr, *M = nullptr, *V = nullptr;
    uint16_t *W1b = nullptr, *W2b = nullptr, *W3b = nullptr;
    long t = 0;                          // Adam steps taken
    long cap = 0;                        // rows of the activation buffers
    float *Z1 = nullptr, *Z2 = nullptr, *Y = nullptr, *dY = nullptr, *dZ2 = nullptr, *dZ1 = nullptr;
    uint16_t *H1 = nullptr, *H2 = nullptr, *dYb = nullptr, *dZ2b = nullptr, *dZ1b = nullptr;
    double *part = nullptr, *dloss = nullptr;
    float *cpart = nullptr;              // column-sum chunk partials
    float *kpart = nullptr;              // split-K partial products
    long cpart_cap = 0, kpart_cap = 0;
    // training staging
    long bcap = 0;
    uint16_t *Xb = nullptr;
    float *Tb = nullptr;
    int64_t *idx = nullptr;
    long idx_cap = 0;
};
