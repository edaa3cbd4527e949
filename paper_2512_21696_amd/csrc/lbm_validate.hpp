// Host-only validation helpers (no device calls).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "../../include/lbm.h"

namespace lbm {
int validate_tables(const lbm_pore_table *t, int ntab, char *msg, size_t len);
int validate_geometry(long long N, const uint8_t *cls, const double *phi, const uint8_t *pt,
                      int ntab, char *msg, size_t len);
int validate_densities(long long N, const uint8_t *cls, const double *rw, const double *ro,
                       int ncomp, char *msg, size_t len);
}  // namespace lbm
