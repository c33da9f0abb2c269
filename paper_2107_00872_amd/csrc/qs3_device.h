// Device helpers of the combinatorial-number-system basis (Sec. 3.1) and of
// the translation representatives (Sec. 3.3), written for gfx950: K = N_down
// is a template constant so that a state lives in K registers, binomial
// columns are read from LDS, and every loop over the K down spins unrolls.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace qs3 {

// Compile-time loop m = M..K-1 (the hop code needs m as a constant).
template <int M, int K>
struct StaticFor {
    template <typename F>
    __host__ __device__ __forceinline__ static void run(F &&f) {
        f(std::integral_constant<int, M>{});
        StaticFor<M + 1, K>::run(f);
    }
};
template <int K>
struct StaticFor<K, K> {
    template <typename F>
    __host__ __device__ __forceinline__ static void run(F &&) {}
};

// ---------------------------------------------------------------------------
// Binomial columns C(c, m) for m = 2..K, c = 0..N, stored column after column
// (entry (m-2)*(N+1) + c); C(c, 1) = c needs no table and C(c, m) = 0 for
// c < m is stored as such.  RT is uint32_t when C(N, K) < 2^32, else uint64_t.
template <typename RT>
struct Binom {
    const RT *tab;
    int sh;  // column m starts at (m - 2) << sh (2^sh > N, so an index is a shift and an add)
    __host__ __device__ __forceinline__ RT C(int c, int m) const {
        return m == 1 ? (RT)c : tab[((m - 2) << sh) + c];
    }
};

// log2 of the binomial column stride for N sites: the smallest 2^sh > N.
__host__ __device__ __forceinline__ int binom_shift(int N) {
    int sh = 0;
    while ((1 << sh) <= N) ++sh;
    return sh;
}

// Unrank (Sec. 3.1, the inverse of Eq. (a_of_n); Alg. 1 with 0-based ranks):
// for m = K..2 the largest c in [m-1, hi] with C(c, m) <= r, then c_1 = r.
// The search is a fixed-trip branch-free bisection so that lanes stay
// converged.
template <int K, typename RT>
__host__ __device__ __forceinline__ void unrank(RT r, int N, const Binom<RT> &B, int (&c)[K > 0 ? K : 1]) {
    int hi = N - 1;
    const int top = 1 << (31 - __builtin_clz((unsigned)N));
#pragma unroll
    for (int m = K; m >= 2; --m) {
        int pos = m - 1;
        for (int step = top; step > 0; step >>= 1) {
            int cand = pos + step;
            if (cand <= hi && B.C(cand, m) <= r) pos = cand;
        }
        c[m - 1] = pos;
        r -= B.C(pos, m);
        hi = pos - 1;
    }
    if (K >= 1) c[0] = (int)r;
}

template <int K, typename RT>
__host__ __device__ __forceinline__ RT rank_of(const int (&c)[K > 0 ? K : 1], const Binom<RT> &B) {
    RT r = 0;
#pragma unroll
    for (int t = 0; t < K; ++t) r += B.C(c[t], t + 1);
    return r;
}

// Per-row precomputation for re-ranking after a hop (the spin exchange of
// Alg. 3 without re-sorting): with B_t = C(c_t, t+1), a hop c_m -> j lands on
//   rank' = R - B_m + C(j, p+1) + sum_{t<m, c_t>j} (C(c_t,t+2) - B_t)
//                             + sum_{t>m, c_t<j} (C(c_t,t)   - B_t),
// p = #{t != m : c_t < j}; modular arithmetic in RT keeps it exact.
template <int K, typename RT>
struct HopRanker {
    RT Bt[K > 0 ? K : 1], dU[K > 0 ? K : 1], dD[K > 0 ? K : 1];
    __host__ __device__ __forceinline__ void init(const int (&c)[K > 0 ? K : 1], const Binom<RT> &B) {
#pragma unroll
        for (int t = 0; t < K; ++t) {
            Bt[t] = B.C(c[t], t + 1);
            dU[t] = (t + 2 <= K) ? (RT)(B.C(c[t], t + 2) - Bt[t]) : (RT)0;
            dD[t] = (t >= 1) ? (RT)(B.C(c[t], t) - Bt[t]) : (RT)0;
        }
    }
    // returns false if j is occupied (no hop); else the new rank in *out
    template <int M>
    __host__ __device__ __forceinline__ bool hop(const int (&c)[K > 0 ? K : 1], RT R, int j, const Binom<RT> &B,
                                        RT *out) const {
        bool down = false;
        int p = 0;
        RT corr = 0;
#pragma unroll
        for (int t = 0; t < K; ++t) {
            if (t == M) continue;
            down |= (c[t] == j);
            bool lt = c[t] < j;
            p += lt ? 1 : 0;
            if (t < M) corr += lt ? (RT)0 : dU[t];
            else corr += lt ? dD[t] : (RT)0;
        }
        *out = R - Bt[M] + corr + B.C(j, p + 1);
        return !down;
    }
    // the same with a run-time spin index m (branch-free selects)
    __host__ __device__ __forceinline__ bool hop_rt(int m, const int (&c)[K > 0 ? K : 1], RT R, int j,
                                                    const Binom<RT> &B, RT *out) const {
        bool down = false;
        int p = 0;
        RT corr = 0, bm = 0;
#pragma unroll
        for (int t = 0; t < K; ++t) {
            const bool self = t == m;
            const bool lt = c[t] < j;
            down |= !self && (c[t] == j);
            p += (!self && lt) ? 1 : 0;
            corr += self ? (RT)0 : (t < m ? (lt ? (RT)0 : dU[t]) : (lt ? dD[t] : (RT)0));
            bm = self ? Bt[t] : bm;
        }
        *out = R - bm + corr + B.C(j, p + 1);
        return !down;
    }
};

// ---------------------------------------------------------------------------
// Lattice geometry for translations.  coords[i] packs the cell coordinates
// and the place in the cell of site i = s + ns * (x + lx * (y + ly * z)):
// x | y<<10 | z<<20 | s<<30.  Translations move cells and keep s.
struct Geom {
    int lx, ly, lz, lxy;
    const uint32_t *coords;
    int ns;
};

__host__ __device__ __forceinline__ int wrap_add(int a, int b, int L) {
    int s = a + b;
    return s >= L ? s - L : s;
}

// Sorting network on K registers (ascending).
template <int K>
__host__ __device__ __forceinline__ void sortK(int (&a)[K > 0 ? K : 1]) {
#pragma unroll
    for (int pass = 0; pass < K; ++pass) {
#pragma unroll
        for (int i = (pass & 1); i + 1 < K; i += 2) {
            int lo = a[i] < a[i + 1] ? a[i] : a[i + 1], hi = a[i] < a[i + 1] ? a[i + 1] : a[i];
            a[i] = lo;
            a[i + 1] = hi;
        }
    }
}

// The representative of the orbit of the sorted tuple c (Sec. 3.3: the minimum
// rank over all translations) and a translation t with T^t c = rep.  The rank
// order is colex, i.e. tuples compare from their largest element down, and an
// image of minimum rank has cell coordinate 0 occupied along every axis
// (otherwise shifting that axis by -1 lowers every index by ns), so only the
// shifts that move
// some down spin to coordinate 0 on each axis are candidates: K^D images
// instead of the N of Alg. 7.
template <int K>
__host__ __device__ __forceinline__ void canonicalize(const int (&c)[K > 0 ? K : 1], const Geom &g,
                                             int (&best)[K > 0 ? K : 1], int &btx, int &bty,
                                             int &btz) {
    int x[K > 0 ? K : 1], y[K > 0 ? K : 1], z[K > 0 ? K : 1], sb[K > 0 ? K : 1];
#pragma unroll
    for (int m = 0; m < K; ++m) {
        uint32_t p = g.coords[c[m]];
        x[m] = p & 1023u;
        y[m] = (p >> 10) & 1023u;
        z[m] = (p >> 20) & 1023u;
        sb[m] = (int)(p >> 30);
        best[m] = c[m];
    }
    btx = bty = btz = 0;
    const int nx = g.lx > 1 ? K : 1, ny = g.ly > 1 ? K : 1, nz = g.lz > 1 ? K : 1;
    for (int iz = 0; iz < nz; ++iz) {
        int tz = z[iz] == 0 ? 0 : g.lz - z[iz];
        for (int iy = 0; iy < ny; ++iy) {
            int ty = y[iy] == 0 ? 0 : g.ly - y[iy];
            for (int ix = 0; ix < nx; ++ix) {
                int tx = x[ix] == 0 ? 0 : g.lx - x[ix];
                int img[K > 0 ? K : 1];
#pragma unroll
                for (int m = 0; m < K; ++m)
                    img[m] = sb[m] + g.ns * (wrap_add(x[m], tx, g.lx) + g.lx * wrap_add(y[m], ty, g.ly) +
                                             g.lxy * wrap_add(z[m], tz, g.lz));
                sortK<K>(img);
                // colex comparison from the top
                int cmp = 0;
#pragma unroll
                for (int m = K - 1; m >= 0; --m)
                    if (cmp == 0) cmp = (img[m] < best[m]) ? -1 : (img[m] > best[m] ? 1 : 0);
                if (cmp < 0) {
#pragma unroll
                    for (int m = 0; m < K; ++m) best[m] = img[m];
                    btx = tx;
                    bty = ty;
                    btz = tz;
                }
            }
        }
    }
}

// Index of `key` in the ascending representative list reps[0..n) through the
// directory dir (dir[b] = first index with reps >= b << shift).
__host__ __device__ __forceinline__ int64_t find_rep(const uint64_t *__restrict__ reps,
                                            const uint32_t *__restrict__ dir, int shift,
                                            uint64_t key) {
    uint64_t b = key >> shift;
    int64_t lo = dir[b], hi = dir[b + 1];  // answer in [lo, hi)
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) >> 1;
        if (reps[mid] <= key) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t n) {
    // gfx950 dispatches workgroup b to XCD b % 8; give each XCD one contiguous
    // slice of the logical block range so its L2 sees neighbouring rows.
    return (n % 8u == 0u) ? (b % 8u) * (n / 8u) + b / 8u : b;
}

// Packed structure-table entry: union index (32 bits) | tx | ty<<10 | tz<<20 (<<32).
__host__ __device__ __forceinline__ uint64_t pack_ent(uint32_t u, int tx, int ty, int tz) {
    return (uint64_t)u | ((uint64_t)(tx | (ty << 10) | (tz << 20)) << 32);
}

// Bit 62 of a hop-list entry marks a target representative with a
// non-trivial stabiliser (its size and k-compatibility have to be read);
// decoders mask the translation to its three 10-bit fields, and bit 63 is
// clear in every entry, so ~0 still marks an empty slot.
constexpr uint64_t HOP_NT_BIT = 1ull << 62;

// SplitMix64 (Steele, Lea, Flood 2014), output `counter` of the stream `seed`.
__host__ __device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t counter) {
    uint64_t z = seed + (counter + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__host__ __device__ __forceinline__ double u01_pm1(uint64_t z) {
    return 2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
}

}  // namespace qs3
