// Placeholders for executors not built yet.
#include "kernels.hpp"
namespace pcot {
bool tiled1d_supported(const int*) { return false; }
hipError_t launch_tiled1d(int, const int*, const TiledLaunch&, int, hipStream_t) { return hipErrorInvalidValue; }
bool tiled3d_supported(const int*) { return false; }
hipError_t launch_tiled3d(int, const int*, const TiledLaunch&, int, hipStream_t) { return hipErrorInvalidValue; }
}
