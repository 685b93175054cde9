// Host-side symbolic plan of the supernodal factorization and the device
// task tables built from it.  Internal to the library.
#pragma once

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace spx {

constexpr int32_t kMaxWidth = 256;  // widest column block handled by the device kernels

struct InvalidArgument : std::runtime_error {
    explicit InvalidArgument(const std::string& s) : std::runtime_error(s) {}
};

struct Options {
    int32_t leaf_size = 64;
    int32_t amalg_pct = 12;
    int32_t split_width = 256;
    const int32_t* user_perm = nullptr;
    bool lu = false;   // L U: device maps for both triangles (assembly into the L and U^T panels)
};

struct Plan {
    int32_t n = 0, ncblk = 0, nblok = 0, nsnode = 0, nsn_fund = 0;
    int64_t nnz_a = 0, nnz_exact = 0, nnz_stored = 0, zeros_used = 0, panel_entries = 0;
    double flops_alg = 0.0, flops_exec = 0.0;         // L L^T and L D L^T: sum of squared column counts
    double flops_alg_lu = 0.0, flops_exec_lu = 0.0;   // L U: sum of 2 (eta - 1)^2 + (eta - 1)
    std::vector<int32_t> perm, iperm, etree, snptr;
    std::vector<int32_t> fcol, lcol, stride, bptr, cparent, uptr, utgt, dep, col_cblk;
    std::vector<int64_t> panel_off;
    std::vector<int32_t> frow, lrow, fcblk, coefind;
    // device maps
    std::vector<int64_t> amap;            // input entry -> panel offset, -1 if not read
                                          // (L U: offsets >= panel_entries are in the U^T panels)
    std::vector<int64_t> rptr;            // symmetric residual pattern (row pointers)
    std::vector<int32_t> rcol;            //   column of each entry
    std::vector<int64_t> rval;            //   index of its value in the input array
};

void analyze_pattern(int32_t n, const int64_t* colptr, const int32_t* rowind, const Options& opt, Plan& P);
void build_device_maps(const int64_t* colptr, const int32_t* rowind, Plan& P, bool lu);
int32_t panel_row(const Plan& P, int32_t k, int32_t r);

}  // namespace spx
