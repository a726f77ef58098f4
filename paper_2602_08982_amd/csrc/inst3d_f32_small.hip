// Instantiation unit of the full-3D kernel set (float; shapes listed below).
#include "engine3d.h"

namespace tdslda {
std::unique_ptr<Engine> make3d_f32_small(int nx, int ny, int nz) {
  if (nx == 4 && ny == 4 && nz == 4) return std::unique_ptr<Engine>(new Engine3D<float, 4, 4, 4>());
  if (nx == 6 && ny == 6 && nz == 6) return std::unique_ptr<Engine>(new Engine3D<float, 6, 6, 6>());
  if (nx == 8 && ny == 8 && nz == 8) return std::unique_ptr<Engine>(new Engine3D<float, 8, 8, 8>());
  if (nx == 8 && ny == 8 && nz == 16) return std::unique_ptr<Engine>(new Engine3D<float, 8, 8, 16>());
  if (nx == 12 && ny == 12 && nz == 12) return std::unique_ptr<Engine>(new Engine3D<float, 12, 12, 12>());
  if (nx == 16 && ny == 16 && nz == 16) return std::unique_ptr<Engine>(new Engine3D<float, 16, 16, 16>());
  return nullptr;
}
}  // namespace tdslda
