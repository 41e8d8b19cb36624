// POD on gfx950 (Sec. 4.1): snapshot Gram, FP64 eigensolver, spatial basis
// with re-orthonormalisation, temporal bases with completion.
#include "internal.h"

extern "C" size_t st_build_bases_workspace(int64_t N_s, int32_t N_t, int32_t n_mu, int32_t n_s, const int32_t* n_t,
                                           int32_t gram_prec) {
  (void)N_s; (void)N_t; (void)n_mu; (void)n_s; (void)n_t; (void)gram_prec;
  return 0;
}

extern "C" st_status st_build_bases(const void* U, int32_t U_prec, int64_t ldU, int64_t N_s, int32_t N_t, int32_t n_mu,
                                    int32_t n_s, const int32_t* n_t, int32_t gram_prec, double tau_t, double* Phi_s,
                                    double* Phi_t, double* sigma, int32_t* rank_t, void* ws, size_t ws_bytes,
                                    void* stream) {
  (void)U; (void)U_prec; (void)ldU; (void)N_s; (void)N_t; (void)n_mu; (void)n_s; (void)n_t; (void)gram_prec;
  (void)tau_t; (void)Phi_s; (void)Phi_t; (void)sigma; (void)rank_t; (void)ws; (void)ws_bytes; (void)stream;
  return ST_EUNSUPPORTED;
}
