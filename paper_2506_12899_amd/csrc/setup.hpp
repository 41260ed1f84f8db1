// Host setup entry points (see setup.cpp).
#pragma once

#include <string>
#include <utility>
#include <vector>

#include "common.hpp"

namespace sbm {

int build_level(const Geometry &g, const sbm_options &o, int n, int p, bool finest_mesh, HostLevel &L,
                std::string &err);
// cell blocks D_K, their inverses (with the singular-value floor) of a level
// whose active set, faces and shifts are in place
int build_blocks(HostLevel &L, const sbm_options &o, std::string &err);
void build_transfer(const HostLevel &Lc, HostLevel &Lf);
void embedding_1d(const HostLevel &Lc, const HostLevel &Lf, double P1[2][MAXN1][MAXN1]);
int coarse_matrix(const HostLevel &L, double alpha, int ext, std::vector<double> &A);
bool invert(double *D, int n, double rel_tol, double reg);
void cell_block(const HostLevel &L, double alpha, int ext, int K, double *D);
void coupling_block(const HostLevel &L, int k, int s, double *C);
void make_kref(const HostLevel &L, const sbm_options &o, double omega, KRef<double> &k);

}  // namespace sbm
