// Internal declarations shared by the host preprocessing and the HIP runtime
// side of libfdu.  Not part of the public ABI (include/fdu.h).
#pragma once

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "fdu.h"

namespace fdu {

// Error carried from internal code to the ABI boundary, where it becomes a
// status code plus the thread-local message of fdu_last_error().
struct Error : std::runtime_error {
  fdu_status code;
  Error(fdu_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& msg);

// Runs f() and turns exceptions into a status code.
template <class F>
fdu_status guard(F&& f) {
  try {
    f();
    return FDU_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return FDU_ERR_OOM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return FDU_ERR_INVALID_ARG;
  }
}

}  // namespace fdu

struct fdu_prep {
  int64_t nv_total = 0, nv_real = 0, ne_flux = 0, nnz_v = 0, nnz_e = 0;
  int64_t n_artificial = 0;
  std::vector<int32_t> perm, iperm, flux_edge, sten6, vptr, vcol, eptr, ecol, ghost_src, artificial;
  std::vector<int8_t> ghost_refl;
  std::vector<double> geo, wfg, we, hmin;
};
