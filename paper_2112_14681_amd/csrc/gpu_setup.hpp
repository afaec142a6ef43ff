// Device construction of the AMG hierarchy (PMIS coarsening and BAMG direct interpolation, Section 5.1),
// gpu_setup.hip. Plain C++ declarations, callable from host-only translation units.
#pragma once

#include "../../include/namg.h"
#include "setup_host.hpp"

namespace namg {

// The hierarchy of p with coarsen = NAMG_COARSEN_PMIS, built level by level on device p.device (seed of
// level l: p.seed + l). Throws SetupError (invalid parameters, zero coarse diagonal) or HipError.
HostHierarchy build_hierarchy_pmis_device(HostCsr &&A, const namg_setup_params &p);

}  // namespace namg
