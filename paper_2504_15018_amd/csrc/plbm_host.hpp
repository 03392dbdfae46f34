// Internal host-side declarations of libplbm.
#pragma once

#include "plbm.h"
#include "plbm_device.hpp"

namespace plbm {

// Record a message for plbm_last_error and return code.
int set_error(int code, const char* fmt, ...);

// Parameter layer (plbm_params.cpp).
double params_K_from_width(double xi, double rho_v, double rho_l);
double params_kappa_from_gamma(double gamma, double K, double rho_v, double rho_l);
int params_resolve(const plbm_phys_params* phys, const plbm_lattice_map* map, plbm_lattice_params* out);
int params_pr_lattice(double T_over_Tc, double omega, double eps, double kappa, double tau_v, double tau_l,
                      const double* body_force, plbm_lattice_params* out);
int params_paper_lattice(double rho_v, double rho_l, double xi, double eps, double kappa, double tau_v,
                         double tau_l, const double* body_force, plbm_lattice_params* out);
double params_gamma_over_kappa(const plbm_lattice_params* p);

}  // namespace plbm
