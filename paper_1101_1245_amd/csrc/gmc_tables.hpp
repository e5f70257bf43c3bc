// gmc_tables.hpp -- host-side table construction for the transport kernels.
#pragma once
#include <vector>

#include "gmc_internal.hpp"
#include "gpumcd.h"

namespace gmc {

struct HostTables {
  int n_mat = 0;
  std::vector<float4> ph;   // [n_mat][kNE] {mu_C, mu_C + mu_pe, mu_total, 0}
  std::vector<float4> el;   // [n_mat][kNE] {L, Sigma_M, Sigma_B, 1/lambda_1}
  std::vector<float> ms;    // [kNms] ln A at logit(G1)
  double ms_y0 = 0.0, ms_dy = 1.0;
};

// Tables for n_mat materials with Moller threshold kcut and bremsstrahlung
// threshold kc (MeV), evaluated in double precision and stored as FP32.
void build_tables(const gmc_material* mats, int n_mat, double kcut, double kc, HostTables* out);

// Majorants per grid bin for a phantom whose densest voxel of material m has
// density rho_max[m] (0 when absent): `margin` times the photon total
// attenuation and the electron hard-event cross section at either bin edge,
// the latter as a running maximum over lower bins.
void build_majorants(const HostTables& t, const double* rho_max, double margin, float* maj_g, float* maj_e);

}  // namespace gmc
