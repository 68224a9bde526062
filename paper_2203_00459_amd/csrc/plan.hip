// Plan-time tables: the transpose of the polar gather as a CSR matrix.
//
// The polar samples sit at fixed frequencies u(b, a) for a given (n, n_r,
// n_theta), so the map from sample (b, a) to the half-plane bins its bilinear
// read touches (Cart2Pol, with the |F(-k)| = |F(k)| fold) is the same for
// every pair.  A device kernel evaluates the corners and weights with the very
// arithmetic of the forward gather (polar_uv, floor, weights), the host groups
// them by bin in sample order, and the adjoint gathers dA = Cart2Pol^T dP with
// one pass over each bin's row: deterministic, no atomics.  Bins outside the
// band-pass get empty rows (the adjoint multiplies their dA by 0 anyway).
#include <vector>

#include "internal.hpp"

namespace fmbym {

__global__ void k_polar_corners(const float2* __restrict__ tw, int n, int n_r, int n_theta,
                                int* __restrict__ bin, float* __restrict__ wgt) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_r * n_theta) return;
    const int b = s / n_theta, a = s % n_theta;
    float uy, ux;
    polar_uv(tw, n, n_r, n_theta, b, a, uy, ux);
    const float fy = floorf(uy), fx = floorf(ux);
    const float wy = uy - fy, wx = ux - fx;
    const int y0 = (int)fy, x0 = (int)fx;
    const int H1 = n / 2 + 1;
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
            int ky = y0 + dy, kx = x0 + dx;
            if (kx < 0) {
                ky = -ky;
                kx = -kx;
            }
            ky &= (n - 1);
            bin[4 * s + 2 * dy + dx] = ky * H1 + kx;
            wgt[4 * s + 2 * dy + dx] = (dy ? wy : 1.f - wy) * (dx ? wx : 1.f - wx);
        }
}

int build_polar_csr(Plan& pl) {
    const int n = pl.p.n, n_r = pl.p.n_r, nt = pl.p.n_theta;
    const int ns = n_r * nt, nbins = n * (n / 2 + 1);
    int* d_bin = nullptr;
    float* d_w = nullptr;
    hipError_t e = hipMalloc((void**)&d_bin, sizeof(int) * 4 * (size_t)ns);
    if (e == hipSuccess) e = hipMalloc((void**)&d_w, sizeof(float) * 4 * (size_t)ns);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_polar_corners, dim3((ns + 255) / 256), dim3(256), 0, 0, pl.twiddle, n, n_r,
                           nt, d_bin, d_w);
        e = hipGetLastError();
    }
    std::vector<int> bin(4 * (size_t)ns);
    std::vector<float> w(4 * (size_t)ns);
    if (e == hipSuccess) e = hipMemcpy(bin.data(), d_bin, sizeof(int) * bin.size(), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(w.data(), d_w, sizeof(float) * w.size(), hipMemcpyDeviceToHost);
    if (d_bin) (void)hipFree(d_bin);
    if (d_w) (void)hipFree(d_w);
    if (e != hipSuccess) return (int)e;
    // bins outside the band-pass get empty rows: their dA is multiplied by 0
    const int h1 = n / 2 + 1;
    auto in_band = [&](int b) {
        if (!pl.band_on) return true;
        const int ky = b / h1, kx = b % h1;
        const int kys = ky < n / 2 ? ky : ky - n;
        const int r2 = kys * kys + kx * kx;
        return r2 >= pl.band_lo2 && r2 <= pl.band_hi2;
    };
    for (size_t i = 0; i < bin.size(); ++i)
        if (!in_band(bin[i])) w[i] = 0.f;
    // Row order: 16 x 16 tiles of the bins kx < n/2 (tile rows outer), then
    // the column kx = n/2.  A block of 256 consecutive rows covers one tile,
    // whose polar samples form a compact patch of the (r, theta) grid, so the
    // adjoint's gather reads whole cache lines of dP.
    std::vector<int> order;
    order.reserve(nbins);
    for (int ty = 0; ty < n / kDmagTile; ++ty)
        for (int tx = 0; tx < (n / 2) / kDmagTile; ++tx)
            for (int y = 0; y < kDmagTile; ++y)
                for (int x = 0; x < kDmagTile; ++x)
                    order.push_back((ty * kDmagTile + y) * h1 + tx * kDmagTile + x);
    for (int ky = 0; ky < n; ++ky) order.push_back(ky * h1 + n / 2);
    std::vector<int> rank(nbins), dst(nbins);
    for (int q = 0; q < nbins; ++q) {
        rank[order[q]] = q;
        dst[q] = (order[q] / h1) * pitch_mag(n) + order[q] % h1;
    }
    // counting sort by row; entries of one row stay in sample order
    std::vector<int> ptr(nbins + 1, 0);
    for (size_t i = 0; i < bin.size(); ++i)
        if (w[i] != 0.f) ++ptr[rank[bin[i]] + 1];
    for (int i = 0; i < nbins; ++i) ptr[i + 1] += ptr[i];
    const int nnz = ptr[nbins];
    std::vector<int> col(nnz);
    std::vector<float> val(nnz);
    std::vector<int> fill(ptr.begin(), ptr.end() - 1);
    for (size_t i = 0; i < bin.size(); ++i) {
        if (w[i] == 0.f) continue;
        const int k = fill[rank[bin[i]]]++;
        col[k] = (int)(i / 4);      // sample index b * n_theta + a
        val[k] = w[i];
    }
    // Blocks of the adjoint: runs of consecutive rows, at most kDmagRows rows
    // and kDmagChunk entries each (a longer single row gets a block alone), so
    // the dense rows near the centre do not pile up in one block.
    std::vector<int> part{0};
    for (int r = 0; r < nbins;) {
        int r1 = r + 1;
        while (r1 < nbins && r1 - r < kDmagRows && ptr[r1 + 1] - ptr[r] <= kDmagChunk) ++r1;
        part.push_back(r1);
        r = r1;
    }
    pl.dmag_nparts = (int)part.size() - 1;
    e = hipMalloc((void**)&pl.csr_ptr, sizeof(int) * ptr.size());
    if (e == hipSuccess) e = hipMalloc((void**)&pl.csr_col, sizeof(int) * (nnz > 0 ? nnz : 1));
    if (e == hipSuccess) e = hipMalloc((void**)&pl.csr_val, sizeof(float) * (nnz > 0 ? nnz : 1));
    if (e == hipSuccess) e = hipMalloc((void**)&pl.csr_dst, sizeof(int) * nbins);
    if (e == hipSuccess) e = hipMemcpy(pl.csr_ptr, ptr.data(), sizeof(int) * ptr.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc((void**)&pl.dmag_part, sizeof(int) * part.size());
    if (e == hipSuccess) e = hipMemcpy(pl.csr_dst, dst.data(), sizeof(int) * nbins, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(pl.dmag_part, part.data(), sizeof(int) * part.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && nnz)
        e = hipMemcpy(pl.csr_col, col.data(), sizeof(int) * nnz, hipMemcpyHostToDevice);
    if (e == hipSuccess && nnz)
        e = hipMemcpy(pl.csr_val, val.data(), sizeof(float) * nnz, hipMemcpyHostToDevice);
    return (int)e;
}

}  // namespace fmbym
