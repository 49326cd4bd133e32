// Face exchange of an x-slab shard: the one-GPU part of the paper's domain
// decomposition with halo regions (Sec. 2.1.1: every stencil kernel reads a
// halo populated from the neighbouring sub-domains; Sec. 5: the decomposed
// runs).  A shard owns planes 0 .. nx-1 of a lattice split along x; its time
// levels also hold halo planes -2, -1 and nx, nx+1 (F, G) and -1, nx (phi_c),
// which the single-pass step reads in place of a periodic wrap.
//
// What the step at plane 0 reads from below: the f and g populations moving
// +x out of plane -1 (pulls into plane 0), and every population that forms
// phi at plane -1 (its stencil neighbour): g with c_x = 0 at plane -1, g with
// c_x = +1 at plane -2 and, with FP32 storage, phi_c of plane -1.  (The g
// with c_x = -1 come from plane 0, the shard's own.)  Mirror images above.
// One face buffer carries exactly that, 24 component planes of ny*nz values
// of the storage type in site order y*nz + z, then (FP32 storage) the plane
// of phi_c words:
//   slots 0..4    f_i with c_x = s of the boundary plane
//   slots 5..18   g_i with c_x in {0, s} of the boundary plane
//   slots 19..23  g_i with c_x = s of the plane behind it (one further in)
// with s = +1 for the face sent up (boundary plane nx-1, behind it nx-2;
// stored by the receiver as its planes -1 and -2) and s = -1 for the face
// sent down (planes 0 and 1; stored as the receiver's nx and nx+1).  A
// periodic lattice on one GPU is the shard that receives its own faces.
#include "lb_device.h"

namespace lbk {

using namespace dev;

namespace {

constexpr int kFaceSlots = 24;

// component of slot k for direction sign s (index order within each group)
__device__ __forceinline__ int face_comp(int k, int s, bool* is_f, bool* behind)
{
    *is_f = k < 5;
    *behind = k >= 19;
    const int want_f = k < 5 ? k : (k >= 19 ? k - 19 : -1);  // rank among c_x = s
    const int want_g = k - 5;                                 // rank among c_x in {0, s}
    int rf = 0, rg = 0;
#pragma unroll
    for (int i = 0; i < NV; i++) {
        if (CX[i] == s) {
            if (rf == want_f) return i;
            rf++;
        }
        if (k >= 5 && k < 19 && (CX[i] == 0 || CX[i] == s)) {
            if (rg == want_g) return i;
            rg++;
        }
    }
    return 0;
}

// pack = true: buffer <- level (boundary plane xb, behind it xb - s);
// pack = false: level <- buffer (into halo planes xb and xb - s).
template <typename T, bool REF>
__global__ __launch_bounds__(kBlock) void k_face(KParams p, T* __restrict__ F, T* __restrict__ G,
                                                 unsigned* __restrict__ phic, T* __restrict__ buf,
                                                 int s, int xb, int pack)
{
    const int a = p.ny * p.nz;
    const int yz = blockIdx.x * kBlock + threadIdx.x;
    const int k = blockIdx.y;
    if (yz >= a) return;
    const int y = yz / p.nz, z = yz - y * p.nz;
    if (k == kFaceSlots) {
        if (!REF) return;
        unsigned* pb = reinterpret_cast<unsigned*>(buf + size_t(kFaceSlots) * a);
        const int c = phic_site(p, xb, y, z);
        if (pack) pb[yz] = phic[c];
        else phic[c] = pb[yz];
        return;
    }
    bool is_f, behind;
    const int i = face_comp(k, s, &is_f, &behind);
    T* arr = is_f ? F : G;
    const unsigned d = didx(p, i, behind ? xb - s : xb, y, z);
    T* b = buf + size_t(k) * a + yz;
    if (pack) *b = arr[d];
    else arr[d] = *b;
}

}  // namespace

size_t face_bytes(const KParams& p, bool fp32)
{
    const size_t a = size_t(p.ny) * p.nz;
    const size_t b = fp32 ? (kFaceSlots + 1) * a * 4 : kFaceSlots * a * 8;
    return (b + 255) / 256 * 256;
}

hipError_t launch_face(const KParams& p, bool fp32, void* state, void* buf, int s, int xb,
                       bool pack, hipStream_t st)
{
    const int a = p.ny * p.nz;
    const dim3 grid((a + kBlock - 1) / kBlock, kFaceSlots + (fp32 ? 1 : 0));
    if (fp32) {
        Lvl<float> l = level<float>(state, p, true);
        k_face<float, true><<<grid, kBlock, 0, st>>>(p, l.F, l.G, l.phic, static_cast<float*>(buf),
                                                     s, xb, pack ? 1 : 0);
    } else {
        Lvl<double> l = level<double>(state, p, false);
        k_face<double, false><<<grid, kBlock, 0, st>>>(p, l.F, l.G, nullptr,
                                                       static_cast<double*>(buf), s, xb,
                                                       pack ? 1 : 0);
    }
    return hipGetLastError();
}

}  // namespace lbk
