// Error reporting shared by the C-ABI source files.
#pragma once

#include <string>

#include "cpi.h"

namespace cpi {
// Records msg as the calling thread's last error (cpi_last_error) and returns s.
cpi_status report_error(cpi_status s, const std::string& msg);
}  // namespace cpi
