// rs_snapshot.hip -- checkpoint and resume of a batch's state.
//
// The state of a batch is its pose, goal, step and episode arrays: the stream
// is counter based (keyed by env id and stream time), so these arrays are all
// that a bit-identical resume needs. A snapshot is a host buffer: a 32-byte
// header, then x, y, theta, goal_x, goal_y ([R] values of the batch's
// precision each) and step, episode ([E] int32 each).
#include "rs_internal.hpp"

#include <cstring>

namespace rs {

namespace {

struct SnapHeader {
  char magic[8];  // "RSSNAP1"
  int32_t dtype;
  int32_t num_envs;
  int64_t robots_total;
  int64_t reserved;
};
static_assert(sizeof(SnapHeader) == 32, "snapshot header is 32 bytes");

constexpr char kMagic[8] = {'R', 'S', 'S', 'N', 'A', 'P', '1', '\0'};

int64_t value_bytes(int32_t dtype) { return dtype == RS_F64 ? 8 : 4; }

rs_status check_snapshot_args(rs_ctx *ctx, int32_t dtype, const rs_batch *b, int64_t robots_total,
                              const void *host, int64_t bytes) {
  RS_CHECK_ARG(ctx != nullptr && b != nullptr && host != nullptr, "ctx/batch/host is NULL");
  RS_CHECK_ARG(dtype == RS_F32 || dtype == RS_F64, "dtype must be RS_F32 or RS_F64");
  RS_CHECK_ARG(b->num_envs >= 1 && robots_total >= 2 * (int64_t)b->num_envs,
               "num_envs >= 1 and robots_total >= 2 * num_envs required");
  RS_CHECK_ARG(b->x && b->y && b->theta && b->goal_x && b->goal_y && b->step && b->episode,
               "state pointer is NULL");
  const int64_t need = rs_snapshot_bytes(dtype, b->num_envs, robots_total);
  RS_CHECK_ARG(bytes >= need, "snapshot buffer holds %lld bytes, %lld needed", (long long)bytes,
               (long long)need);
  return RS_OK;
}

}  // namespace

}  // namespace rs

using namespace rs;

extern "C" {

int64_t rs_snapshot_bytes(int32_t dtype, int32_t num_envs, int64_t robots_total) {
  if (num_envs < 0 || robots_total < 0) return 0;
  return (int64_t)sizeof(SnapHeader) + 5 * robots_total * value_bytes(dtype) +
         2 * (int64_t)num_envs * 4;
}

rs_status rs_snapshot(rs_ctx *ctx, int32_t dtype, const rs_batch *b, int64_t robots_total,
                      void *host, int64_t bytes, void *stream) {
  rs_status s = check_snapshot_args(ctx, dtype, b, robots_total, host, bytes);
  if (s != RS_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  char *out = static_cast<char *>(host);
  SnapHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, kMagic, sizeof(kMagic));
  h.dtype = dtype;
  h.num_envs = b->num_envs;
  h.robots_total = robots_total;
  std::memcpy(out, &h, sizeof(h));
  char *p = out + sizeof(h);
  const size_t rb = (size_t)(robots_total * value_bytes(dtype));
  const void *fields[5] = {b->x, b->y, b->theta, b->goal_x, b->goal_y};
  for (const void *f : fields) {
    RS_CHECK_HIP(hipMemcpyAsync(p, f, rb, hipMemcpyDeviceToHost, st));
    p += rb;
  }
  const size_t eb = (size_t)b->num_envs * 4;
  RS_CHECK_HIP(hipMemcpyAsync(p, b->step, eb, hipMemcpyDeviceToHost, st));
  RS_CHECK_HIP(hipMemcpyAsync(p + eb, b->episode, eb, hipMemcpyDeviceToHost, st));
  RS_CHECK_HIP(hipStreamSynchronize(st));
  return RS_OK;
}

rs_status rs_restore(rs_ctx *ctx, int32_t dtype, const rs_batch *b, int64_t robots_total,
                     const void *host, int64_t bytes, void *stream) {
  rs_status s = check_snapshot_args(ctx, dtype, b, robots_total, host, bytes);
  if (s != RS_OK) return s;
  const char *in = static_cast<const char *>(host);
  SnapHeader h;
  std::memcpy(&h, in, sizeof(h));
  RS_CHECK_ARG(std::memcmp(h.magic, kMagic, sizeof(kMagic)) == 0, "not a snapshot buffer");
  RS_CHECK_ARG(h.dtype == dtype && h.num_envs == b->num_envs && h.robots_total == robots_total,
               "snapshot of (dtype %d, %d envs, %lld robots) does not match the batch",
               h.dtype, h.num_envs, (long long)h.robots_total);
  hipStream_t st = (hipStream_t)stream;
  const char *p = in + sizeof(h);
  const size_t rb = (size_t)(robots_total * value_bytes(dtype));
  void *fields[5] = {b->x, b->y, b->theta, b->goal_x, b->goal_y};
  for (void *f : fields) {
    RS_CHECK_HIP(hipMemcpyAsync(f, p, rb, hipMemcpyHostToDevice, st));
    p += rb;
  }
  const size_t eb = (size_t)b->num_envs * 4;
  RS_CHECK_HIP(hipMemcpyAsync(b->step, p, eb, hipMemcpyHostToDevice, st));
  RS_CHECK_HIP(hipMemcpyAsync(b->episode, p + eb, eb, hipMemcpyHostToDevice, st));
  RS_CHECK_HIP(hipStreamSynchronize(st));
  return RS_OK;
}

}  // extern "C"
