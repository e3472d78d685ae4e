// Device-side local least-squares reconstruction of a moving triangulated
// surface (connectivity built once on the host, cached until it changes).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ib {

struct SurfMesh {
    int nv = 0, ne = 0;
    uint64_t hash = 0;
    int32_t* ring_ptr = nullptr;   // two-ring CSR (itself included, ascending)
    int32_t* ring = nullptr;
    int32_t* vt_ptr = nullptr;     // vertex -> 3 t + corner of its triangles (ascending)
    int32_t* vt = nullptr;
    int32_t* tri = nullptr;        // the triangles (device copy of the validated host ones)
    double* Xa = nullptr;          // advanced vertices
    double* n0 = nullptr;          // their angle-weighted normals
    int* flag = nullptr;
    void release();
    // (re)builds the connectivity when nv, ne or the triangles (host) change
    int prepare(int nv, int ne, const int32_t* T_host);
    // X + dt U moved onto the fitted surface: Xo, fs (sigma kappa), ds, nrm (device).
    // Syncs (degenerate-neighbourhood flag).
    int reconstruct(const double* X, const double* U, double dt, double sigma, double* Xo, double* fs,
                    double* ds, double* nrm, hipStream_t st);
};

}  // namespace ib
