// Instantiation unit of the full-3D kernel set (double; shapes listed below).
#include "engine3d.h"

namespace tdslda {
std::unique_ptr<Engine> make3d_f64_large(int nx, int ny, int nz) {
  if (nx == 24 && ny == 24 && nz == 24) return std::unique_ptr<Engine>(new Engine3D<double, 24, 24, 24>());
  if (nx == 32 && ny == 32 && nz == 32) return std::unique_ptr<Engine>(new Engine3D<double, 32, 32, 32>());
  if (nx == 48 && ny == 48 && nz == 48) return std::unique_ptr<Engine>(new Engine3D<double, 48, 48, 48>());
  return nullptr;
}
}  // namespace tdslda
