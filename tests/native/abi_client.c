/* A plain C client of libsu2.so: no PyTorch, no C++.  It allocates the
 * lattice with the HIP runtime, runs a hot start, two steps of 1 heat-bath
 * + 1 overrelaxation sweep, the plaquette and the Polyakov loop through the
 * C ABI of include/su2.h, and prints them, so that a GPU test can check the
 * boundary is usable on its own (and gives the values the Python binding
 * gives).  Usage: abi_client Nx Ny Nz Nt prec(0 f64, 1 f32) beta seed */
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "su2.h"

static int check(int rc, const char *what)
{
    if (rc != SU2_OK) {
        fprintf(stderr, "%s: %s (%s)\n", what, su2_strerror(rc), su2_last_error());
        exit(1);
    }
    return rc;
}

int main(int argc, char **argv)
{
    if (argc != 8) {
        fprintf(stderr, "usage: %s Nx Ny Nz Nt prec beta seed\n", argv[0]);
        return 2;
    }
    su2_lattice_t lat;
    for (int k = 0; k < 4; ++k)
        lat.n[k] = atoi(argv[1 + k]);
    lat.prec = atoi(argv[5]);
    lat.lattice_id = 0;
    lat.tile = 0;
    lat.tile_y = 0;
    const double beta = atof(argv[6]);
    const uint64_t seed = strtoull(argv[7], NULL, 10);
    const uint64_t lb = su2_links_bytes(lat.n, lat.prec), wb = su2_workspace_bytes(lat.n, lat.prec);
    if (lb == 0 || wb == 0) {
        fprintf(stderr, "invalid lattice\n");
        return 1;
    }
    double *d_obs = NULL;
    if (hipMalloc(&lat.links, lb) != hipSuccess || hipMalloc(&lat.work, wb) != hipSuccess ||
        hipMalloc((void **)&d_obs, 9 * sizeof(double)) != hipSuccess) {
        fprintf(stderr, "hipMalloc failed\n");
        return 1;
    }
    lat.work_bytes = wb;
    hipStream_t st;
    if (hipStreamCreate(&st) != hipSuccess)
        return 1;
    check(su2_init_hot(&lat, seed, st), "su2_init_hot");
    for (uint32_t s = 0; s < 2; ++s) {
        check(su2_heatbath_sweep(&lat, beta, seed, s, st), "su2_heatbath_sweep");
        check(su2_overrelax(&lat, 1, st), "su2_overrelax");
    }
    check(su2_plaquette(&lat, d_obs, st), "su2_plaquette");
    check(su2_polyakov(&lat, d_obs + 7, NULL, st), "su2_polyakov");
    uint32_t *d_flags = NULL, flags = 0;
    if (hipMalloc((void **)&d_flags, sizeof(uint32_t)) != hipSuccess)
        return 1;
    check(su2_get_flags(&lat, d_flags, st), "su2_get_flags");
    double obs[9];
    if (hipStreamSynchronize(st) != hipSuccess ||
        hipMemcpy(obs, d_obs, sizeof obs, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(&flags, d_flags, sizeof flags, hipMemcpyDeviceToHost) != hipSuccess) {
        fprintf(stderr, "copy back failed\n");
        return 1;
    }
    printf("plaquette %.17g\npolyakov %.17g %.17g\nflags %u\n", obs[0], obs[7], obs[8], flags);
    hipFree(lat.links);
    hipFree(lat.work);
    hipFree(d_obs);
    hipFree(d_flags);
    hipStreamDestroy(st);
    return 0;
}
