// Solve-phase layouts packed on the device from device-built levels (pack.hip).
#pragma once

#include "device.hpp"

namespace namg {

// False when NAMG_HOST_PACK is set: device-built hierarchies are then packed on the host like the others
// (the two paths give the same bytes; the switch lets tests compare them).
bool device_packing_enabled();

// M packed from the device CSR D exactly as DMat::build packs the same matrix from a host CSR (layout
// choice, 16/32-bit columns, values cast to T; a prolongation in the unit-row layout `unit` when it applies;
// the slice-diagonal form only when allow_dia). Runs on the null stream and waits for it.
template <class T>
void pack_device(DMat<T> &M, const DCsr &D, MemCounter *mc, int force_group = 0, const UnitRows *unit = nullptr,
                 bool allow_dia = true);

// The polynomial Gauss-Seidel data of level matrix A: lo = D^{-1}L, up = D^{-1}U (FP64, a_ij / a_ii),
// dinv = 1 / a_ii and dl1inv = 1 / sum_j |a_ij| (as T), with the host setup's arithmetic.
template <class T>
void smoother_data_device(const DCsr &A, DCsr &lo, DCsr &up, DevBuf<T> &dinv, DevBuf<T> &dl1inv, MemCounter *mc);

extern template void pack_device<float>(DMat<float> &, const DCsr &, MemCounter *, int, const UnitRows *, bool);
extern template void pack_device<double>(DMat<double> &, const DCsr &, MemCounter *, int, const UnitRows *, bool);
extern template void smoother_data_device<float>(const DCsr &, DCsr &, DCsr &, DevBuf<float> &, DevBuf<float> &,
                                                 MemCounter *);
extern template void smoother_data_device<double>(const DCsr &, DCsr &, DCsr &, DevBuf<double> &,
                                                  DevBuf<double> &, MemCounter *);

}  // namespace namg
