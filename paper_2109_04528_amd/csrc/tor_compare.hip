// tor_compare.hip -- the comparison kernels: a fresh factorisation per
// subset (Algorithm 1) and the removal order of Sec. 2 (Algorithm 2).  They
// are not the method; they measure it against the forms the paper describes.
#include "tor_device.hpp"
#include "tor_internal.hpp"

namespace tor {

// ---------------------------------------------------------------------------
// Comparison baseline: a fresh factorisation per subset (Algorithm 1 applied
// to each (I-O)_Z independently, two rows at a time), one wave per subset.
// S = double runs it on the real quadrature form (a Gaussian-state matrix, as
// the recursive kernel does), S = c64 on the complex matrix.
constexpr int PLAIN_MAX_N = 34;

template <class S>
__global__ void __launch_bounds__(64) tor_plain(PlainParams prm)
{
    __shared__ S A[E(PLAIN_MAX_N)];
    __shared__ S vec[4 * 2 * PLAIN_MAX_N];
    __shared__ int rows[2 * PLAIN_MAX_N];
    __shared__ uint16_t xy[E(PLAIN_MAX_N)];  // packed entry e -> row x << 8 | column y
    const int lane = threadIdx.x;
    const int n = prm.n, N = prm.N;
    const S *C = reinterpret_cast<const S *>(prm.C);
    // the (x, y) of every packed lower-triangle entry, once: the gather and
    // the updates below then look them up instead of walking the triangle
    for (int e = lane; e < E(n); e += 64) {
        int x, y;
        block_ab(e, x, y);
        xy[e] = (uint16_t)((x << 8) | y);
    }
    AccDD acc;
    int bad = 0;
    for (;;) {
        const unsigned long long c = bcast_first(atomicAdd(prm.counter, lane == 0 ? 1ull : 0ull));
        const unsigned long long z0 = prm.mask_begin + c * (unsigned long long)prm.chunk;
        if (z0 >= prm.mask_end)
            break;
        unsigned long long z1 = z0 + prm.chunk;
        if (z1 > prm.mask_end)
            z1 = prm.mask_end;
        for (unsigned long long Z = z0; Z < z1; ++Z) {
            const int d = __popcll(Z);
            // reversed interleaved rows of (I-O)_Z in terms of the staged
            // matrix: lane r < d finds the r-th highest mode of Z
            if (lane < d) {
                unsigned long long zz = Z;
                for (int q = 0; q < lane; ++q)
                    zz &= ~(1ull << (63 - __clzll(zz)));
                const int m = 63 - __clzll(zz);
                rows[2 * lane] = 2 * N - 2 - 2 * m;
                rows[2 * lane + 1] = 2 * N - 1 - 2 * m;
            }
            __syncthreads();
            const int ed = E(d);
            for (int e = lane; e < ed; e += 64) {
                const int x = xy[e] >> 8, y = xy[e] & 0xff;
                const int gx = rows[x], gy = rows[y];  // gx >= gy
                A[e] = blk(C, NB(N), bidx(gx >> 1, gy >> 1), ((gx & 1) << 1) + (gy & 1));
            }
            __syncthreads();
            double det = 1.0;
            for (int s = d; s >= 1; --s) {
                const int p = 2 * s - 2;
                const double a = re(A[pidx(p, p)]);
                const S b = A[pidx(p + 1, p)];
                const double g = re(A[pidx(p + 1, p + 1)]);
                Piv<S> pv = pivot(a, b, g);
                if (!(a > 0.0) || !(pv.pdet > 0.0))
                    bad = 1;
                det *= pv.pdet;
                if (s == 1)
                    break;
                for (int y = lane; y < p; y += 64) {
                    S r1 = A[pidx(p, y)];
                    S r2 = sub_mul(A[pidx(p + 1, y)], r1, pv.ba);
                    vec[y] = scale(r1, pv.inv_a);
                    vec[p + y] = r1;
                    vec[2 * p + y] = scale(r2, pv.inv_g);
                    vec[3 * p + y] = r2;
                }
                __syncthreads();
                const int eo = p * (p + 1) / 2;
                for (int e = lane; e < eo; e += 64) {
                    const int x = xy[e] >> 8, y = xy[e] & 0xff;
                    S v = upd(A[e], vec[x], vec[p + y], vec[2 * p + x], vec[3 * p + y]);
                    A[e] = (x == y) ? fix_diag(v) : v;
                }
                __syncthreads();
            }
            if (lane == 0) {
                const double t = rsqrt_nr(det);
                if ((n - d) & 1)
                    acc.template add<-1>(t);
                else
                    acc.template add<1>(t);
            }
            __syncthreads();
        }
    }
    const int anybad = __any(bad);
    if (lane == 0) {
        double *o = prm.partials + 4 * blockIdx.x;
        o[0] = acc.hi;
        o[1] = acc.lo;
        o[2] = acc.abs_sum;
        o[3] = anybad ? 1.0 : 0.0;
    }
}

// ---------------------------------------------------------------------------
// The removal order of Sec. 2 (Algorithm 2), as a comparison kernel.  A node
// is the set of kept modes; its child removes one mode i larger than every
// mode removed so far, keeps the rows and columns of the kept modes below i
// and the rows of the modes above i restricted to those columns (L11, L21),
// and factorises the trailing block afresh: L22 = chol(C22 - L21 L21^H), a
// scalar Cholesky of the matrix of the modes above i (Algorithm 1).  The
// determinant is the product of the squared diagonal.
//
// Storage per wave (global scratch): one level per depth of the walk; level L
// holds the rows of the modes above its removed mode (the root level: every
// kept mode).  The row pair of mode q sits at NSZ(q) with 2q + 2 entries per
// row (its kept rank r <= q needs 2r + 1 or 2r + 2), so a child's rows are at
// the same offsets as its parent's.  A child reads only its parent's rows
// (the rows above i, which the parent level holds) and writes its own.
// pref[L][q]: product of the squared diagonal of the rows of the kept modes
// <= q in the node of level L (valid for q >= that level's removed mode).
__device__ __forceinline__ int roff(int q) { return 2 * q * (q + 1); }

// Cholesky in place of rows rowoff[0..M2) of a level buffer, columns c0 + y
// (y <= x); piv[j] receives the j-th squared diagonal entry.
__device__ void removal_factor(c64 *lev, const int *rowoff, int c0, int M2, double *piv, int lane, int &bad)
{
    for (int j = 0; j < M2; ++j) {
        const double dj = lev[rowoff[j] + c0 + j].x;
        if (!(dj > 0.0))
            bad = 1;
        const double ljj = sqrt(dj);
        const double inv = 1.0 / ljj;
        __syncthreads();
        if (lane == 0) {
            piv[j] = dj;
            lev[rowoff[j] + c0 + j] = c64{ljj, 0.0};
        }
        for (int x = j + 1 + lane; x < M2; x += 64) {
            c64 &e = lev[rowoff[x] + c0 + j];
            e = c64{e.x * inv, e.y * inv};
        }
        __syncthreads();
        const int w = M2 - 1 - j;
        for (int t = lane; t < w * (w + 1) / 2; t += 64) {
            int xx, yy;
            block_ab(t, xx, yy);
            const int x = j + 1 + xx, y = j + 1 + yy;
            const c64 a = lev[rowoff[x] + c0 + j], b = lev[rowoff[y] + c0 + j];
            c64 &e = lev[rowoff[x] + c0 + y];
            // e -= a conj(b)
            const double er = e.x - (a.x * b.x + a.y * b.y);
            const double ei = e.y - (a.y * b.x - a.x * b.y);
            e = c64{er, x == y ? 0.0 : ei};
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(64) tor_removal(RemovalParams prm)
{
    constexpr int NM = REMOVAL_MAX_N;
    __shared__ int rowoff[2 * NM];
    __shared__ int modeOf[NM];
    __shared__ double piv[2 * NM];
    __shared__ double pref[(NM + 1) * NM];
    __shared__ int next[NM + 1];
    const int lane = threadIdx.x;
    const int n = prm.n, k = prm.k;
    const c64 *C = reinterpret_cast<const c64 *>(prm.C);
    c64 *scr = reinterpret_cast<c64 *>(prm.scratch + (long long)blockIdx.x * prm.scratch_stride);
    const int LV = NSZ(n);  // scalars per level
    AccDD acc;
    int bad = 0;
    for (;;) {
        const unsigned long long root = bcast_first(atomicAdd(prm.counter, lane == 0 ? 1ull : 0ull));
        if (root >= (1ull << k))
            break;
        const int nrem0 = __popcll(root);
        const int nk = n - nrem0;
        // root node: a fresh factorisation of the kept modes
        for (int q = lane; q < n; q += 64) {
            const bool rem = q < k && ((root >> q) & 1ull);
            if (!rem) {
                const int r = q - __popcll(root & ((1ull << q) - 1ull));
                modeOf[r] = q;
            }
        }
        __syncthreads();
        for (int x = lane; x < 2 * nk; x += 64) {
            const int q = modeOf[x >> 1];
            rowoff[x] = roff(q) + (x & 1) * (2 * q + 2);
        }
        __syncthreads();
        for (int t = lane; t < nk * (2 * nk + 1); t += 64) {
            int x, y;
            block_ab(t, x, y);
            const int gx = 2 * modeOf[x >> 1] + (x & 1), gy = 2 * modeOf[y >> 1] + (y & 1);
            c64 v = C[pidx(gx, gy)];
            if (x == y)
                v.y = 0.0;
            scr[rowoff[x] + y] = v;
        }
        __syncthreads();
        removal_factor(scr, rowoff, 0, 2 * nk, piv, lane, bad);
        if (lane == 0) {
            double pr = 1.0;
            int r = 0;
            for (int q = 0; q < n; ++q) {
                const bool rem = q < k && ((root >> q) & 1ull);
                if (!rem) {
                    pr *= piv[2 * r] * piv[2 * r + 1];
                    ++r;
                }
                pref[q] = pr;
            }
            next[0] = k;
        }
        __syncthreads();
        {
            const double det = n > 0 ? pref[n - 1] : 1.0;
            const double t = rsqrt_nr(det);
            if (lane == 0) {
                if (nrem0 & 1)
                    acc.template add<-1>(t);
                else
                    acc.template add<1>(t);
            }
        }
        // depth-first walk over the removals of the modes k..n-1
        int d = 0;
        for (;;) {
            const int i = next[d];
            __syncthreads();
            if (i >= n) {
                if (d == 0)
                    break;
                --d;
                continue;
            }
            if (lane == 0)
                next[d] = i + 1;
            const int nrem = nrem0 + d;
            const int c = i - nrem;  // kept modes below i
            const int m = n - 1 - i; // modes above i (all kept)
            const c64 *par = scr + (long long)d * LV;
            c64 *chd = scr + (long long)(d + 1) * LV;
            for (int x = lane; x < 2 * m; x += 64) {
                const int q = i + 1 + (x >> 1);
                rowoff[x] = roff(q) + (x & 1) * (2 * q + 2);
            }
            __syncthreads();
            // L21: the parent's rows above i, first 2c columns
            for (int t = lane; t < 2 * m * 2 * c; t += 64) {
                const int x = t / (2 * c), j = t - x * (2 * c);
                chd[rowoff[x] + j] = par[rowoff[x] + j];
            }
            // C22 - L21 L21^H into the trailing block
            for (int t = lane; t < m * (2 * m + 1); t += 64) {
                int x, y;
                block_ab(t, x, y);
                const int gx = 2 * (i + 1) + x, gy = 2 * (i + 1) + y;
                c64 v = C[pidx(gx, gy)];
                const c64 *px = par + rowoff[x], *py = par + rowoff[y];
                for (int j = 0; j < 2 * c; ++j) {
                    const c64 a = px[j], b = py[j];
                    v.x -= a.x * b.x + a.y * b.y;
                    v.y -= a.y * b.x - a.x * b.y;
                }
                if (x == y)
                    v.y = 0.0;
                chd[rowoff[x] + 2 * c + y] = v;
            }
            __syncthreads();
            removal_factor(chd, rowoff, 2 * c, 2 * m, piv, lane, bad);
            if (lane == 0) {
                double *pp = pref + (d + 1) * NM;
                double pr = i > 0 ? pref[d * NM + i - 1] : 1.0;
                pp[i] = pr;
                for (int q = i + 1; q < n; ++q) {
                    const int t2 = 2 * (q - i - 1);
                    pr *= piv[t2] * piv[t2 + 1];
                    pp[q] = pr;
                }
                next[d + 1] = i + 1;
            }
            __syncthreads();
            const double det = pref[(d + 1) * NM + n - 1];
            const double t = rsqrt_nr(det);
            if (lane == 0) {
                if ((nrem + 1) & 1)
                    acc.template add<-1>(t);
                else
                    acc.template add<1>(t);
            }
            ++d;
        }
    }
    const int anybad = __any(bad);
    if (lane == 0) {
        double *o = prm.partials + 4 * blockIdx.x;
        o[0] = acc.hi;
        o[1] = acc.lo;
        o[2] = acc.abs_sum;
        o[3] = anybad ? 1.0 : 0.0;
    }
}

__global__ void __launch_bounds__(64) tor_plain_reduce(const double *parts, int nwaves, double *out)
{
    const int lane = threadIdx.x;
    double h = 0.0, l = 0.0, ab = 0.0, bad = 0.0;
    for (int w = lane; w < nwaves; w += 64) {
        dd_add2(h, l, parts[4 * w], parts[4 * w + 1]);
        ab += parts[4 * w + 2];
        bad = fmax(bad, parts[4 * w + 3]);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        double oh = __shfl_xor(h, off), ol = __shfl_xor(l, off);
        dd_add2(h, l, oh, ol);
        ab += __shfl_xor(ab, off);
        bad = fmax(bad, __shfl_xor(bad, off));
    }
    if (lane == 0) {
        out[0] = h;
        out[1] = l;
        out[2] = ab;
        out[3] = bad;
    }
}

// ---------------------------------------------------------------------------
hipError_t launch_plain(const PlainParams &p, bool real, int grid, hipStream_t s)
{
    if (real)
        hipLaunchKernelGGL((tor_plain<double>), dim3(grid), dim3(64), 0, s, p);
    else
        hipLaunchKernelGGL((tor_plain<c64>), dim3(grid), dim3(64), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_removal(const RemovalParams &p, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(tor_removal, dim3(grid), dim3(64), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_plain_reduce(const double *partials, int nwaves, double *result, hipStream_t s)
{
    hipLaunchKernelGGL(tor_plain_reduce, dim3(1), dim3(64), 0, s, partials, nwaves, result);
    return hipGetLastError();
}

}  // namespace tor
