// Host-side state of one lattice (the opaque lbm_ctx of include/lbm.h).  Shared by
// the single-lattice calls and the batched form; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/lbm.h"
#include "lbm_internal.hpp"

struct lbm_ctx {
    lbm_lattice lat;
    lbm_eos eos;
    lbm_params p;
    double derived[27];
    lbm_dev::Consts<double> c64;
    lbm_dev::Consts<float> c32;
    const void* consts;       // &c64 or &c32 depending on precision
    lbm_dev::Walls<double> w64;   // boundary state of a LBM_BC_HEATED_OUTFLOW lattice
    lbm_dev::Walls<float> w32;
    const void* walls;        // &w64 or &w32
    bool host_only;
    void* ws;
    size_t ws_bytes;
    hipStream_t stream;
    void* buf[2];
    size_t state_bytes;
    double* rho_scratch;
    double* partials;
    double* result;
    int cur;
    bool fields_set;
    int64_t steps;
    lbm_dev::LaunchShape shape;
    std::string err;
};
