// k_frame.hip -- frame driver: camera rays, first-collision delta tracking,
// compaction of the hits into a point list, and the image write.
//
// These kernels produce the shading points a frame queries (they are support
// for the hot path, not part of the method).  One ray per pixel: pinhole rays
// through pixel centres (row 0 at the top) or orthographic rays along -z
// through the pixel centres of the unit square.  Delta tracking (Woodcock)
// runs on the piecewise-constant voxel density of the finest level with
// majorant sigma_t * max(rho): free flights -log(1-u)/majorant, a tentative
// collision accepted with probability mu/majorant.  Uniform numbers are a
// counter-based hash of (seed, pixel, draw) with the SplitMix64 mixer of
// Steele, Lea and Flood (2014): mix(x) = finalise(x + 0x9E3779B97F4A7C15)
// with xor-shift-multiply rounds (30, 0xBF58476D1CE4E5B9; 27,
// 0x94D049BB133111EB; 31), h = mix(mix(mix(seed) ^ pixel) ^ draw),
// u = (h >> 11) * 2^-53; draw 2i is the i-th flight, 2i+1 its acceptance.
// Geometry runs in double precision.  The hit flags are compacted through an
// exclusive prefix sum: wavefront prefix sums within blocks of 1024 flags,
// then one workgroup scans the block totals (and writes the hit count), and
// the compaction adds each block's prefix.
#include "launch_args.h"

namespace nis {

__device__ __forceinline__ uint64_t sm_mix(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double uniform01(uint64_t seed, uint64_t stream, uint64_t draw)
{
    const uint64_t h = sm_mix(sm_mix(sm_mix(seed) ^ stream) ^ draw);
    return (double)(h >> 11) * (1.0 / 9007199254740992.0);
}

// slab interval of the ray against [0,1]^3; an axis whose products are NaN
// (origin on a face with a zero direction) does not constrain the ray
__device__ __forceinline__ void box_interval(const double o[3], const double d[3], double& t_in, double& t_out)
{
#pragma clang fp contract(off)
    double tmin = -INFINITY, tmax = INFINITY;
    bool any_min = false, any_max = false;
    for (int a = 0; a < 3; a++) {
        const double inv = 1.0 / d[a];
        const double t0 = (0.0 - o[a]) * inv, t1 = (1.0 - o[a]) * inv;
        if (isnan(t0) || isnan(t1)) continue;
        const double lo = t0 < t1 ? t0 : t1, hi = t0 < t1 ? t1 : t0;
        tmin = any_min ? fmax(tmin, lo) : lo;
        tmax = any_max ? fmin(tmax, hi) : hi;
        any_min = any_max = true;
    }
    t_in = fmax(tmin, 0.0);
    t_out = tmax;
}

__device__ __forceinline__ void camera_ray(const CamArgs& C, int px, int py, double o[3], double d[3])
{
#pragma clang fp contract(off)
    if (C.ortho) {
        o[0] = (px + 0.5) / C.width;
        o[1] = (py + 0.5) / C.height;
        o[2] = C.oz;
        d[0] = 0.0;
        d[1] = 0.0;
        d[2] = -1.0;
        return;
    }
    const double col = (px + 0.5) / C.width * 2.0 - 1.0;
    const double row = 1.0 - (py + 0.5) / C.height * 2.0;
    const double sc = col * C.aspect * C.tan_half, sr = row * C.tan_half;
    for (int a = 0; a < 3; a++) {
        o[a] = C.eye[a];
        d[a] = (C.f[a] + sc * C.r[a]) + sr * C.u[a];
    }
    const double nrm = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
    for (int a = 0; a < 3; a++) d[a] /= nrm;
}

// Pixel of ray slot s.  In bands of B rows (the last band may be lower) the
// slots walk each band column by column, so that consecutive collisions, and
// the shading points that run side by side on a compute unit, form compact
// patches of the image rather than strips of one row.
__device__ __forceinline__ int64_t slot_pixel(int64_t s, int w, int h, int band)
{
    if (band <= 1) return s;
    const int64_t full = (int64_t)band * w;
    const int64_t b = s / full, r = s - b * full;
    const int64_t hb = (int64_t)h - b * band < band ? (int64_t)h - b * band : band;
    return (b * band + r % hb) * w + r / hb;
}

__global__ void __launch_bounds__(256)
k_raygen(CamArgs C, const float* __restrict__ rho, int n, double sigma_t, double majorant, uint64_t seed,
         int* __restrict__ flag, float* __restrict__ pts, float* __restrict__ dirs)
{
#pragma clang fp contract(off)
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= (int64_t)C.width * C.height) return;
    const int64_t pix = slot_pixel(slot, C.width, C.height, C.band);
    const int px = (int)(pix % C.width), py = (int)(pix / C.width);
    double o[3], d[3];
    camera_ray(C, px, py, o, d);
    double t_in, t_out;
    box_interval(o, d, t_in, t_out);
    int hit = 0;
    double t = t_in;
    if (t_in < t_out && majorant > 0.0) {
        for (int step = 0; step < kMaxTrackingSteps; step++) {
            const double uf = uniform01(seed, (uint64_t)pix, 2 * (uint64_t)step);
            const double ua = uniform01(seed, (uint64_t)pix, 2 * (uint64_t)step + 1);
            t = t - log1p(-uf) / majorant;
            if (!(t < t_out)) break;
            int idx[3];
            for (int a = 0; a < 3; a++) {
                const double x = o[a] + t * d[a];
                const double fl = floor(x * n);
                idx[a] = fl < 0.0 ? 0 : (fl > n - 1 ? n - 1 : (int)fl);
            }
            const double r = rho[((int64_t)idx[2] * n + idx[1]) * n + idx[0]];
            if (ua * majorant < sigma_t * r) {
                hit = 1;
                break;
            }
        }
    }
    flag[slot] = hit;
    for (int a = 0; a < 3; a++) {
        pts[3 * slot + a] = hit ? (float)(o[a] + t * d[a]) : 0.f;
        dirs[3 * slot + a] = (float)d[a];
    }
}

constexpr int kScanBlock = 1024;   // flags per workgroup of the local scan (256 lanes x 4)

// inclusive prefix sum of v over the 64 lanes of a wavefront
__device__ __forceinline__ int wave_inclusive_scan(int v, int lane)
{
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(v, o);
        if (lane >= o) v += y;
    }
    return v;
}

// Exclusive prefix sum of the flags within each block of kScanBlock slots,
// and each block's total in part[block].
__global__ void __launch_bounds__(256)
k_scan_local(const int* __restrict__ flag, int64_t n, int* __restrict__ offset, int* __restrict__ part)
{
    __shared__ int wsum[4];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + 4 * t;
    int v[4];
    if (base + 3 < n) {
        const int4 f = *reinterpret_cast<const int4*>(flag + base);
        v[0] = f.x, v[1] = f.y, v[2] = f.z, v[3] = f.w;
    } else {
        for (int e = 0; e < 4; e++) v[e] = base + e < n ? flag[base + e] : 0;
    }
    const int s = v[0] + v[1] + v[2] + v[3];
    const int inc = wave_inclusive_scan(s, lane);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int wpre = 0;
    for (int i = 0; i < w; i++) wpre += wsum[i];
    int ex = wpre + inc - s;
    for (int e = 0; e < 4; e++) {
        if (base + e < n) offset[base + e] = ex;
        ex += v[e];
    }
    if (t == 255) part[blockIdx.x] = wpre + inc;
}

// Exclusive prefix sum of the nb block totals in place (one workgroup, each
// lane a contiguous run of them), and the total: the frame's hit count.
__global__ void __launch_bounds__(1024) k_scan_parts(int* __restrict__ part, int nb, int* __restrict__ count)
{
    __shared__ int wsum[16];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int per = (nb + 1023) / 1024;
    const int b0 = min(t * per, nb), b1 = min(b0 + per, nb);
    int s = 0;
    for (int b = b0; b < b1; b++) s += part[b];
    const int inc = wave_inclusive_scan(s, lane);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int wpre = 0;
    for (int i = 0; i < w; i++) wpre += wsum[i];
    int ex = wpre + inc - s;
    for (int b = b0; b < b1; b++) {
        const int v = part[b];
        part[b] = ex;
        ex += v;
    }
    if (t == 1023) *count = wpre + inc;
}

__global__ void __launch_bounds__(256)
k_compact(const int* __restrict__ flag, const int* __restrict__ offset, const int* __restrict__ part,
          const float* __restrict__ pts, const float* __restrict__ dirs, int w, int h, int band,
          float* __restrict__ cpts, float* __restrict__ cdirs, int* __restrict__ cpix)
{
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= (int64_t)w * h || !flag[slot]) return;
    const int64_t o = (int64_t)offset[slot] + part[slot / kScanBlock];
    for (int a = 0; a < 3; a++) {
        cpts[3 * o + a] = pts[3 * slot + a];
        cdirs[3 * o + a] = dirs[3 * slot + a];
    }
    cpix[o] = (int)slot_pixel(slot, w, h, band);
}

__global__ void __launch_bounds__(256) k_fill(float* __restrict__ p, int64_t n, float v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void __launch_bounds__(256)
k_scatter_image(const int* __restrict__ cpix, const float* __restrict__ L, const int* __restrict__ count,
                float scale, float* __restrict__ image)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < *count) image[cpix[i]] = scale * L[i];
}

__global__ void __launch_bounds__(256)
k_scatter_image_rgb(const int* __restrict__ cpix, const float* __restrict__ L, const int* __restrict__ count,
                    float s0, float s1, float s2, float* __restrict__ image)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < *count) {
        const int64_t o = (int64_t)cpix[i] * 3;
        image[o] = s0 * L[3 * i];
        image[o + 1] = s1 * L[3 * i + 1];
        image[o + 2] = s2 * L[3 * i + 2];
    }
}

// scan storage: one total per block of kScanBlock flags
hipError_t frame_scan_bytes(int64_t npix, size_t* bytes)
{
    *bytes = (size_t)((npix + kScanBlock - 1) / kScanBlock + 1) * sizeof(int);
    return hipSuccess;
}

hipError_t launch_raygen(const CamArgs& C, const float* rho0, int n, double sigma_t, double majorant,
                         uint64_t seed, const FrameBuffers& fb, hipStream_t s)
{
    const int64_t npix = (int64_t)C.width * C.height;
    const int blocks = (int)((npix + 255) / 256);
    hipLaunchKernelGGL(k_raygen, dim3(blocks), dim3(256), 0, s, C, rho0, n, sigma_t, majorant, seed, fb.flag,
                       fb.pts, fb.dirs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nb = (npix + kScanBlock - 1) / kScanBlock;
    size_t need = 0;
    frame_scan_bytes(npix, &need);
    if (fb.scan_bytes < need || nb > 0x7fffffff) return hipErrorInvalidValue;
    int* part = reinterpret_cast<int*>(fb.scan_tmp);
    hipLaunchKernelGGL(k_scan_local, dim3((int)nb), dim3(256), 0, s, fb.flag, npix, fb.offset, part);
    hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(1024), 0, s, part, (int)nb, fb.count);
    hipLaunchKernelGGL(k_compact, dim3(blocks), dim3(256), 0, s, fb.flag, fb.offset, part, fb.pts, fb.dirs,
                       C.width, C.height, C.band, fb.cpts, fb.cdirs, fb.cpix);
    return hipGetLastError();
}

hipError_t launch_image(const FrameBuffers& fb, int64_t npix, const float* L, float scale, float* image,
                        hipStream_t s)
{
    const int blocks = (int)((npix + 255) / 256);
    hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, s, image, npix, 0.f);
    hipLaunchKernelGGL(k_scatter_image, dim3(blocks), dim3(256), 0, s, fb.cpix, L, fb.count, scale, image);
    return hipGetLastError();
}

hipError_t launch_image_rgb(const FrameBuffers& fb, int64_t npix, const float* L, const float scale[3],
                            float* image, hipStream_t s)
{
    const int64_t nf = 3 * npix;
    hipLaunchKernelGGL(k_fill, dim3((int)((nf + 255) / 256)), dim3(256), 0, s, image, nf, 0.f);
    hipLaunchKernelGGL(k_scatter_image_rgb, dim3((int)((npix + 255) / 256)), dim3(256), 0, s, fb.cpix, L, fb.count,
                       scale[0], scale[1], scale[2], image);
    return hipGetLastError();
}

}  // namespace nis
