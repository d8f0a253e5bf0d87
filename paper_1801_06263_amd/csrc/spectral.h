// Launchers of the per-ray spectral kernels, the fused primal update and
// the D_TPL reduction (spectral.hip).
#pragma once

#include "kernels.h"

namespace osscir {

hipError_t launch_spectral_model(const ScanDesc &sd, const float *p, const float *c, float *chat, float *r,
                                 float *G, float *H, float *Hp, bool fp64, hipStream_t st);

// y, qS updated from p (line integrals at the expansion point) and counts c;
// pbar (optional): the line integrals of fbar when they differ from p (inner
// iterations of nested loops).
hipError_t launch_spectral_dual(const ScanDesc &sd, const float *p, const float *c, float *y, float *qS,
                                float lambda, bool clip, bool block, bool fp64, hipStream_t st,
                                const float *pbar = nullptr);

// back-projection of qS fused with the primal step and the extrapolation;
// pack (optional): packed images (launch_pack's layout, borders already
// zero) that receive fbar' for the next forward projection; bp: the split
// back-projection's sums (the workspace's bp region; needed when
// sd.bp_parts > 1).
hipError_t launch_back_primal(const ScanDesc &sd, const float *qS, float *f, float *fbar, float lambda, bool block,
                              void *pack, double *bp, hipStream_t st);

// sigma [4][L], per-ray terms (scratch, 6 or 3 channels) and the pixel
// steps out_img (T^-1 upper triangles or tau).
hipError_t launch_steps(const ScanDesc &sd, const float *G, float lambda, bool block, float *sigma, float *terms,
                        float *out_img, hipStream_t st);

// out = M in for 3-channel maps of npix pixels (M row-major 3x3, in place allowed).
hipError_t launch_material_transform(const double M[9], const float *in, float *out, int npix, hipStream_t st);

int dtpl_partial_count(const ScanDesc &sd);
hipError_t launch_dtpl(const ScanDesc &sd, const float *f, const float *c, float *p_scratch, void *pack,
                       double *partial, double *out, hipStream_t st);

}  // namespace osscir
