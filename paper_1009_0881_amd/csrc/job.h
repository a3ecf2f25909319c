// Device-visible description of one NMF problem at one level of its hierarchy
// (a "job").  Every sweep kernel takes an array of jobs plus, per phase, the
// prefix sum of the jobs' tile counts: block b works on tile b - prefix[i] of
// job i.  A single solve launches with one job; a batch or a serving tick
// launches one grouped kernel per phase over all of its jobs.
#pragma once

#include <cstdint>

namespace nmf {

struct DevState;

struct Job {
    const float *M;      // level matrix, m x n column-major, column stride ldm
    int64_t ldm, m, n;
    int32_t r, rpad;     // rank and rank padded to 16
    int32_t tm;          // A-pass rows per tile (16 or 64)
    int32_t chunks;      // split of the length-m reduction of V^T M
    int64_t chunk;       // rows per chunk (multiple of 16)
    int32_t nA, nC, nF, nG;   // tiles of: A-pass, C-pass (nCx * chunks), W update (4
                              // columns each), Gram kernels (upper 16x16 tiles)
    int32_t nCx;         // 64-column tiles of the C-pass
    int32_t wc, cf;      // C-pass row groups per tile; W-update columns per tile
    int32_t nFb;         // W-update blocks (n / cf; nF counts its 4-column partials)
    int32_t depth, log_cap;
    float *V;            // level factor, m x r column-major
    float *W;            // r x n row-major
    float *Wt;           // n x rpad, transposed and zero-padded copy of W; entry k of row
                         // j at j * rpad + wt_pos(k, rpad / 16) (device_common.h)
    float *A;            // products kept in FP32 (nmf_products): M W^T (m x r, column-major)
    float *C;            //   and V^T M (r x n, row-major)
    double *Ad, *Cd;     // ANLS: the same products in FP64 (taken instead of A / C when set),
                         // the right-hand sides of the NNLS problems
    double *Bd, *Dd;     // W W^T and V^T V (r x r, FP64)
    double *Cp;          // V^T M partials: chunks x (n x r, entry (k, j) at j * r + k),
                         // FP64 (prec 0) or FP32 (prec 1, a float view of the buffer)
    double *Dp;          // V^T V partials: chunks x rpad x rpad (upper 16x16 tiles)
    double *Cr;          // V^T M summed over the chunks (n x r, FP64, layout of one chunk)
                         // by the D-reduction kernel's extra blocks, read by the W
                         // update instead of the partials; null: the W update sums them
    int32_t nCr;         // those extra blocks (256 entries each)
    double *rparts;      // residual partials of the W-update tiles, nF
    int32_t gseg;        // B = W W^T: column segments per upper tile (blocks nG * gseg)
    double *bparts;      // their partial tiles: [tile][segment][256] (gseg > 1)
    const double *normM2;   // ||M_depth||^2
    double *log_rel;
    int32_t *log_depth;
    DevState *st;
    int32_t *hstop;      // host-mapped copy of st->stop, set with it (null: none)
    double tol;
    // BF16 precision mode (prec = 1): operand copies for the MFMA passes.
    // Mbp: A-pass copy of M, K-packed: element (i, j) at
    //      ((i/16 * G + j/8) * 16 + i%16) * 8 + j%8, G = npad / 8, zero padded to
    //      16-row panels and npad columns.
    // Mbc: C-pass copy of M, column-major with column stride mpad (rows >= m zero);
    //      on streaming levels column-panelled instead: element (i, j) at
    //      ((j/16 * (mpad/32) + i/32) * 4 + i%32/8) * 128 + j%16 * 8 + i%8, so the
    //      32 x 16 block of a C-pass K-step is 1 KB contiguous (columns >= n zero).
    // Vb:  V, column-major with stride mpad, rpad columns (k >= r zero).
    // Wb:  W, rpad x npad row-major (k >= r or j >= n zero).
    // mpad = m and npad = n rounded up to 128.
    // The stop test is applied only to FP32 (prec = 0) iterations.
    const uint16_t *Mbp, *Mbc;
    uint16_t *Vb, *Wb;
    int64_t mpad, npad;
    int32_t prec;
    int32_t stream;      // 1: streaming A/C-pass kernels (large BF16 levels): A-pass
                         // tiles of kStreamARows rows, C-pass tiles of 256 columns
    int32_t aks;         // FP32 streaming A-pass: the n-reduction split over aks blocks
                         // per row tile (1: none); the partial rows of A (FP64, aks x
                         // nA tm x rpad) occupy Cp until the second half has used them
};

}  // namespace nmf
