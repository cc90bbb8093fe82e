// Lattice indexing on the device: periodic chain (N = L) and periodic cube (N = L^3,
// site i = x + L (y + L z)); bond 3 i + a joins i and its +a neighbour (Sec. IV lattices).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pa {

// + neighbours (x+1, y+1, z+1) of site i of an L^3 periodic cube
__device__ inline void plus_neighbours3(int i, int L, int nb[3])
{
    const int x = i % L, y = (i / L) % L;
    const int LL = L * L;
    nb[0] = (x + 1 == L) ? i - (L - 1) : i + 1;
    nb[1] = (y + 1 == L) ? i - (LL - L) : i + L;
    nb[2] = (i + LL >= LL * L) ? i + LL - LL * L : i + LL;
}

// Checkerboard site of half-index h in colour c (colour (x + y + z) mod 2), L^3 cube:
// row = y + L z = h / (L/2), x = 2 (h mod L/2) + ((c + y + z) mod 2).
// Writes the site and its six neighbours in the order +x, +y, +z, -x, -y, -z.
template <int L>
__device__ inline int cube_site(int h, int c, int nb[6])
{
    constexpr int H = L / 2;
    constexpr int LL = L * L;
    constexpr int N = L * L * L;
    const int row = h / H;
    const int m = h - row * H;
    const int y = row % L;
    const int z = row / L;
    const int x = 2 * m + ((c + y + z) & 1);
    const int i = x + L * row;
    nb[0] = (x + 1 == L) ? i - (L - 1) : i + 1;
    nb[1] = (y + 1 == L) ? i - (LL - L) : i + L;
    nb[2] = (z + 1 == L) ? i - (N - LL) : i + LL;
    nb[3] = (x == 0) ? i + (L - 1) : i - 1;
    nb[4] = (y == 0) ? i + (LL - L) : i - L;
    nb[5] = (z == 0) ? i + (N - LL) : i - LL;
    return i;
}

// chain: site of half-index h in colour c is 2h + c; neighbours +1, -1
__device__ inline int ring_site(int h, int c, int N, int nb[2])
{
    const int i = 2 * h + c;
    nb[0] = (i + 1 == N) ? 0 : i + 1;
    nb[1] = (i == 0) ? N - 1 : i - 1;
    return i;
}

// 6-bit mask of the couplings at site i that are -1, in neighbour order
// (+x, +y, +z, -x, -y, -z): bit k set iff that bond has J = -1
__device__ inline uint32_t cube_jmask(const int8_t* J, int i, int L)
{
    const int x = i % L, y = (i / L) % L, z = i / (L * L);
    const int LL = L * L, N = LL * L;
    const int mx = (x == 0) ? i + (L - 1) : i - 1;
    const int my = (y == 0) ? i + (LL - L) : i - L;
    const int mz = (z == 0) ? i + (N - LL) : i - LL;
    uint32_t m = 0;
    m |= (J[3 * i + 0] < 0) << 0;
    m |= (J[3 * i + 1] < 0) << 1;
    m |= (J[3 * i + 2] < 0) << 2;
    m |= (J[3 * mx + 0] < 0) << 3;
    m |= (J[3 * my + 1] < 0) << 4;
    m |= (J[3 * mz + 2] < 0) << 5;
    return m;
}

__device__ inline uint32_t ring_jmask(const int8_t* J, int i, int N)
{
    const int m = (i == 0) ? N - 1 : i - 1;
    return (uint32_t)(J[i] < 0) | ((uint32_t)(J[m] < 0) << 1);
}

}  // namespace pa
