// Internal declarations shared by the kernels and the host runtime of
// liblopc.so.  Not part of the public ABI (include/lopc.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lopc {

constexpr uint32_t kChunkBytes = 16384;  // 16 kB chunks (Sec. III-B / IV-C)
constexpr uint32_t kHeaderBytes = 64;
constexpr uint32_t kRecordHeaderBytes = 16;
constexpr uint32_t kMagic = 0x43504F4Cu;  // "LOPC"
constexpr uint32_t kVersion = 1;
constexpr uint64_t kMaxPoints = 0xFFFFFFFFull;  // subbins kept in 32 bits

// Device status bits, OR-ed into Params::status by any kernel.
enum : uint32_t {
  ST_NONFINITE = 1u,
  ST_BOUND = 2u,
  ST_RANGE = 4u,
  ST_FORMAT = 8u,
  ST_CAPACITY = 16u,
  ST_INTERNAL = 32u,
};

// Per-call parameters and results, at the start of the workspace.
struct alignas(256) Params {
  double eb;          // bound as given
  double eps;         // absolute bound applied
  double inv;         // smallest binary64 with inv * eps >= 1
  double winv;        // 1 / inv rounded (only a starting point for walks)
  uint32_t status;    // ST_* bits
  uint32_t ticket;    // chunk ticket counter of the encoder
  uint64_t stream_size;
  uint64_t bins_bytes;
  uint64_t sub_bytes;
  int64_t kmin, kmax;  // order keys of the smallest / largest value
  uint32_t mode;
  uint32_t dtype;
  uint8_t header[64];  // copy of the stream header (read back with Params)
};

// A field as a 3D box (a 2D field d0 x d1 is the box 1 x d0 x d1: the same
// neighbours and the same linear indices).
struct Box {
  int32_t nz, ny, nx;
  uint32_t n;  // points
};

// Repair tiling.
struct Tiling {
  int32_t tz, ty, tx;     // tile extent
  int32_t ntz, nty, ntx;  // tiles per axis
  uint32_t ntiles;
};

// Launchers (lopc_kernels.hip).  All enqueue on `s` and return the HIP
// status of the last launch.
hipError_t launch_minmax(int dtype, const void* x, uint32_t n, double* part,
                         int nblocks, Params* prm, hipStream_t s);
hipError_t launch_params(int dtype, int mode, double eb, const double* part,
                         int nblocks, Params* prm, uint8_t* stream,
                         size_t cap, int ndim, const int64_t* dims,
                         hipStream_t s);
hipError_t launch_quant(int dtype, const void* x, uint32_t n, Params* prm, void* bins,
                        int nblocks, hipStream_t s);
hipError_t launch_tile0(int dtype, const void* x, Box box, Tiling t, const void* bins,
                        uint16_t* mask, uint32_t* sub, uint32_t* stamp,
                        uint32_t* counters, hipStream_t s);
hipError_t launch_repair(Box box, Tiling t, const uint16_t* mask,
                         uint32_t* sub, uint32_t* stamp, uint32_t* counters,
                         uint32_t sweep, hipStream_t s);
hipError_t launch_encode(int dtype, uint32_t n, const void* bins,
                         const uint32_t* sub, uint64_t* lookback,
                         uint32_t* parts, Params* prm, uint8_t* stream,
                         size_t cap, hipStream_t s);
hipError_t launch_sum_parts(const uint32_t* parts, uint32_t nch, Params* prm,
                            hipStream_t s);
hipError_t launch_offsets(const uint8_t* stream, uint32_t nch,
                          uint64_t body_bytes, uint64_t* offsets,
                          Params* prm, hipStream_t s);
hipError_t launch_decode(int dtype, const uint8_t* stream, uint32_t n,
                         const uint64_t* offsets, Params* prm, void* field,
                         hipStream_t s);

}  // namespace lopc
