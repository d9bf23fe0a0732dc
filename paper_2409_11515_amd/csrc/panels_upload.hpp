// Upload of one triangular solve's schedule into a device workspace.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "panels.hpp"

namespace condest {

// Uploads t's arrays on `s` at ws + off[...] (offsets from tri_layout with the
// same K), arms the slice partial slots with the not-yet-solved pattern and
// fills `out` with the device pointers.
int tri_upload(char* ws, const size_t* off, const PanelCsr& t, int K, hipStream_t s, DevTri& out);

}  // namespace condest
