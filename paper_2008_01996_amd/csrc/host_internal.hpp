// Internal host-side declarations shared by the library's translation units.
#pragma once

#include <string>
#include <vector>

#include "stfd.h"

struct stfd_space {
    int nv = 0, ntri = 0, Mx = 0, half_band = 0;
    std::vector<double> xy;       // 2 nv
    std::vector<int> tri;         // 3 ntri
    std::vector<int> dof;         // nv
    std::vector<double> area;     // ntri
    // M_x and A_x on one symmetric pattern (CSR, columns sorted)
    std::vector<int> rowptr, col;
    std::vector<double> valM, valA;
    // M10 (M_x x ntri, CSR)
    std::vector<int> rowptr10, col10;
    std::vector<double> val10;
    // couplings of interior rows to Dirichlet vertices (M_x x nv, CSR over
    // vertex numbers): the columns of M_x and A_x dropped for the boundary
    std::vector<int> rowptrB, colB;
    std::vector<double> valMB, valAB;
    // envelope of the pivot-free LDL^T in blocks of 16: block_reach[c] =
    // the number of 16-row blocks below diagonal block c that its columns'
    // band reaches (every later L entry of those columns, fill included,
    // lies in these blocks; at most ceil(half_band / 16))
    std::vector<int> block_reach;
};

namespace stfd {

// thread-local error message helpers; return the code
int fail(int code, const std::string& msg);
void clear_error();

int assemble_time_impl(int Nt, const double* t, double* At, double* Mt, double* Ct);

}  // namespace stfd
