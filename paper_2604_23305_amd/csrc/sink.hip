// Out-of-core runs: a whole observation simulated in pixel groups, each
// group streamed device -> pinned host -> disk while the next one is
// computed (the paper's RAM manager, section 1; output files, section 2.7).
//
// Pipeline (two device slabs, two pinned host halves):
//   compute stream:  [group g+1 into slab (g+1)%2, after slab_free of g-1]
//   copy stream:     [wait computed g] D2H piece -> half h, event -> ...
//   writer thread:   wait piece event, pwrite to the file, free half h
// Files are NumPy .npy (version 1.0): tod.npy [P][K][T] float32 (pixel
// groups are contiguous slabs of the file), pwv.npy [P][T] float32,
// time.npy [T] float64.
#include <hip/hip_runtime.h>

#include <fcntl.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <cerrno>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/gtod.h"
#include "gtod_internal.h"

namespace {

using namespace gtod;

std::string npy_header(const char* descr, const std::vector<int64_t>& shape) {
  std::string d = std::string("{'descr': '") + descr +
                  "', 'fortran_order': False, 'shape': (";
  for (size_t i = 0; i < shape.size(); ++i) {
    d += std::to_string(shape[i]);
    if (shape.size() == 1 || i + 1 < shape.size()) d += ", ";
  }
  d += "), }";
  const size_t used = 10 + d.size() + 1;
  d.append((64 - used % 64) % 64, ' ');
  d += '\n';
  std::string h("\x93NUMPY\x01\x00", 8);
  h.push_back((char)(d.size() & 0xff));
  h.push_back((char)((d.size() >> 8) & 0xff));
  return h + d;
}

bool write_all(int fd, const char* p, size_t n, int64_t off) {
  while (n > 0) {
    const ssize_t w = pwrite(fd, p, n, off);
    if (w < 0) {
      if (errno == EINTR) continue;
      return false;
    }
    p += w;
    n -= (size_t)w;
    off += w;
  }
  return true;
}

struct Piece {
  int fd;
  int64_t off;
  const char* buf;
  size_t bytes;
  hipEvent_t ready;
  int half;
};

// One thread: waits for each piece's copy event, writes it, frees its half.
class Writer {
 public:
  explicit Writer(int device) : th_([this, device] { run(device); }) {}
  ~Writer() { finish(); }

  void wait_free(int h) {
    std::unique_lock<std::mutex> l(m_);
    cv_free_.wait(l, [&] { return !busy_[h]; });
  }
  void push(const Piece& p) {
    std::lock_guard<std::mutex> l(m_);
    busy_[p.half] = true;
    q_.push_back(p);
    cv_.notify_one();
  }
  // Waits until every queued piece is written and stops the thread.
  void finish() {
    {
      std::lock_guard<std::mutex> l(m_);
      if (stop_) return;
      stop_ = true;
      cv_.notify_one();
    }
    th_.join();
  }
  bool failed() const { return failed_; }
  const std::string& message() const { return msg_; }

 private:
  void run(int device) {
    (void)hipSetDevice(device);
    for (;;) {
      Piece p;
      {
        std::unique_lock<std::mutex> l(m_);
        cv_.wait(l, [&] { return stop_ || !q_.empty(); });
        if (q_.empty()) return;
        p = q_.front();
        q_.pop_front();
      }
      const hipError_t e = hipEventSynchronize(p.ready);
      if (!failed_) {
        if (e != hipSuccess) {
          failed_ = true;
          msg_ = std::string("copy to host: ") + hipGetErrorString(e);
        } else if (!write_all(p.fd, p.buf, p.bytes, p.off)) {
          failed_ = true;
          msg_ = std::string("write: ") + std::strerror(errno);
        }
      }
      std::lock_guard<std::mutex> l(m_);
      busy_[p.half] = false;
      cv_free_.notify_all();
    }
  }

  std::mutex m_;
  std::condition_variable cv_, cv_free_;
  std::deque<Piece> q_;
  bool busy_[2] = {false, false};
  bool stop_ = false;
  bool failed_ = false;
  std::string msg_;
  std::thread th_;
};

}  // namespace

extern "C" gtod_status gtod_simulate_to_disk(gtod_ctx* c, const gtod_job* sig,
                                             const gtod_job* pink,
                                             const gtod_sink_desc* sd, double* stats) {
  if (!c) return GTOD_EINVAL;
  if (!sig || !sd || !sd->dir) return ctx_fail(c, GTOD_EINVAL, "NULL argument");
  if (sig->kind != GTOD_JOB_SIGNAL || sig->t_begin != 0 || sig->t_end != sig->t_total ||
      sig->t_total < 1 || sig->n_pix < 1 || !sig->dphi_rad || !sig->dtheta_rad)
    return ctx_fail(c, GTOD_EINVAL, "signal must be a SIGNAL job over [0, t_total) with pixel offsets");
  if (pink && (pink->kind != GTOD_JOB_PINK || pink->spec_id != sig->spec_id ||
               pink->n_pix != sig->n_pix || pink->t_total != sig->t_total ||
               pink->seed != sig->seed))
    return ctx_fail(c, GTOD_EINVAL, "pink must be a PINK job of the same setup, pixels, length and seed");
  if (sd->flags & ~GTOD_SINK_PWV) return ctx_fail(c, GTOD_EINVAL, "unknown sink flags");
  const int K = ctx_spec_channels(c, sig->spec_id);
  if (K < 0) return ctx_fail(c, GTOD_ENOTFOUND, "unknown spec id");
  if (sd->host_bytes < (2u << 20)) return ctx_fail(c, GTOD_EINVAL, "host_bytes < 2 MiB");
  const bool with_pwv = (sd->flags & GTOD_SINK_PWV) != 0;
  const int64_t T = sig->t_total, P = sig->n_pix;
  const int64_t tod_pp = (int64_t)K * T * 4, pwv_pp = with_pwv ? T * 4 : 0;
  int64_t G = sd->pix_per_group > 0
                  ? std::min<int64_t>(sd->pix_per_group, P)
                  : std::min<int64_t>(P, (int64_t)(sd->device_bytes / (2 * (tod_pp + pwv_pp))));
  if (G < 1 || (uint64_t)(2 * G * (tod_pp + pwv_pp)) > sd->device_bytes)
    return ctx_fail(c, GTOD_EINVAL, "device_bytes does not hold two slabs of one pixel group");
  const int64_t n_groups = (P + G - 1) / G;
  if (hipSetDevice(ctx_device(c)) != hipSuccess)
    return ctx_fail(c, GTOD_EDEVICE, "hipSetDevice failed");
  hipStream_t cs = ctx_sink_stream(c, 0), xs = ctx_sink_stream(c, 1);
  if (!cs || !xs) return ctx_fail(c, GTOD_EDEVICE, "stream creation failed");

  const auto wall0 = std::chrono::steady_clock::now();
  gtod_status st = GTOD_OK;
  std::string emsg;
  float* tod_slab[2] = {nullptr, nullptr};
  float* pwv_slab[2] = {nullptr, nullptr};
  char* host = nullptr;
  hipEvent_t computed[2] = {}, slab_free[2] = {}, piece_ev[2] = {};
  int fd_tod = -1, fd_pwv = -1, fd_time = -1;
  for (int i = 0; i < 2 && st == GTOD_OK; ++i) {
    st = ctx_alloc(c, (void**)&tod_slab[i], (size_t)(G * tod_pp));
    if (st == GTOD_OK && with_pwv) st = ctx_alloc(c, (void**)&pwv_slab[i], (size_t)(G * pwv_pp));
  }
  if (st == GTOD_OK && hipHostMalloc((void**)&host, sd->host_bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    host = nullptr;
    st = ctx_fail(c, GTOD_ENOMEM, "pinned staging allocation failed");
  }
  for (int i = 0; i < 2 && st == GTOD_OK; ++i) {
    if (hipEventCreateWithFlags(&computed[i], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&slab_free[i], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&piece_ev[i], hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      st = ctx_fail(c, GTOD_EDEVICE, "event creation failed");
    }
  }
  // files
  const std::string dir(sd->dir);
  const std::string h_tod = npy_header("<f4", {P, K, T});
  const std::string h_pwv = npy_header("<f4", {P, T});
  const std::string h_time = npy_header("<f8", {T});
  if (st == GTOD_OK) {
    if (mkdir(dir.c_str(), 0755) != 0 && errno != EEXIST) {
      st = GTOD_EIO;
      emsg = "cannot create " + dir + ": " + std::strerror(errno);
    }
  }
  auto open_out = [&](const char* name, int* fd) {
    if (st != GTOD_OK) return;
    const std::string path = dir + "/" + name;
    *fd = open(path.c_str(), O_WRONLY | O_CREAT | O_TRUNC, 0644);
    if (*fd < 0) {
      st = GTOD_EIO;
      emsg = "cannot open " + path + ": " + std::strerror(errno);
    }
  };
  open_out("tod.npy", &fd_tod);
  if (with_pwv) open_out("pwv.npy", &fd_pwv);
  open_out("time.npy", &fd_time);
  if (st == GTOD_OK) {
    const double fs = ctx_f_sample(c);
    std::vector<double> tv((size_t)T);
    for (int64_t n = 0; n < T; ++n) tv[(size_t)n] = (double)n / fs;
    bool ok = write_all(fd_tod, h_tod.data(), h_tod.size(), 0) &&
              write_all(fd_time, h_time.data(), h_time.size(), 0) &&
              write_all(fd_time, (const char*)tv.data(), tv.size() * 8, (int64_t)h_time.size());
    if (ok && with_pwv) ok = write_all(fd_pwv, h_pwv.data(), h_pwv.size(), 0);
    if (!ok) {
      st = GTOD_EIO;
      emsg = std::string("write: ") + std::strerror(errno);
    }
  }

  int64_t bytes = 0;
  if (st == GTOD_OK) {
    const size_t half = (sd->host_bytes / 2) / 4096 * 4096;
    char* hb[2] = {host, host + half};
    Writer wr(ctx_device(c));
    int hnext = 0;
    auto enqueue_group = [&](int64_t g) -> gtod_status {
      const int slot = (int)(g & 1);
      const int64_t p0 = g * G, np = std::min(G, P - p0);
      if (g >= 2 && hipStreamWaitEvent(cs, slab_free[slot], 0) != hipSuccess)
        return ctx_fail(c, GTOD_EDEVICE, "stream wait failed");
      gtod_job js[2];
      int nj = 0;
      if (pink) {
        js[nj] = *pink;
        js[nj].n_pix = (int32_t)np;
        js[nj].pix0 = (int32_t)p0;
        js[nj].tod = tod_slab[slot];
        js[nj].out_t0 = 0;
        js[nj].out_ld = T;
        js[nj].flags &= ~GTOD_JOB_ACCUMULATE;
        ++nj;
      }
      js[nj] = *sig;
      js[nj].n_pix = (int32_t)np;
      js[nj].pix0 = (int32_t)p0;
      js[nj].dphi_rad = sig->dphi_rad + p0;
      js[nj].dtheta_rad = sig->dtheta_rad + p0;
      js[nj].tod = tod_slab[slot];
      js[nj].p_kid = nullptr;
      js[nj].sigma = nullptr;
      js[nj].pwv = with_pwv ? pwv_slab[slot] : nullptr;
      js[nj].out_t0 = 0;
      js[nj].out_ld = T;
      if (pink) js[nj].flags |= GTOD_JOB_ACCUMULATE;
      else js[nj].flags &= ~GTOD_JOB_ACCUMULATE;
      ++nj;
      const gtod_status s2 = gtod_simulate_tod(c, js, nj, cs);
      if (s2 != GTOD_OK) return s2;
      if (hipEventRecord(computed[slot], cs) != hipSuccess)
        return ctx_fail(c, GTOD_EDEVICE, "event record failed");
      return GTOD_OK;
    };
    auto copy_range = [&](int fd, int64_t off, const char* src, int64_t n) -> gtod_status {
      for (int64_t o = 0; o < n; o += (int64_t)half) {
        const size_t m = (size_t)std::min<int64_t>((int64_t)half, n - o);
        const int h = hnext;
        hnext ^= 1;
        wr.wait_free(h);
        if (wr.failed()) return GTOD_EIO;
        if (hipMemcpyAsync(hb[h], src + o, m, hipMemcpyDeviceToHost, xs) != hipSuccess ||
            hipEventRecord(piece_ev[h], xs) != hipSuccess)
          return ctx_fail(c, GTOD_EDEVICE, "copy to host failed");
        wr.push(Piece{fd, off + o, hb[h], m, piece_ev[h], h});
        bytes += (int64_t)m;
      }
      return GTOD_OK;
    };
    auto copy_group = [&](int64_t g) -> gtod_status {
      const int slot = (int)(g & 1);
      const int64_t p0 = g * G, np = std::min(G, P - p0);
      if (hipStreamWaitEvent(xs, computed[slot], 0) != hipSuccess)
        return ctx_fail(c, GTOD_EDEVICE, "stream wait failed");
      gtod_status s2 = copy_range(fd_tod, (int64_t)h_tod.size() + p0 * tod_pp,
                                  (const char*)tod_slab[slot], np * tod_pp);
      if (s2 == GTOD_OK && with_pwv)
        s2 = copy_range(fd_pwv, (int64_t)h_pwv.size() + p0 * pwv_pp,
                        (const char*)pwv_slab[slot], np * pwv_pp);
      if (s2 == GTOD_OK && hipEventRecord(slab_free[slot], xs) != hipSuccess)
        s2 = ctx_fail(c, GTOD_EDEVICE, "event record failed");
      return s2;
    };
    st = enqueue_group(0);
    for (int64_t g = 0; g < n_groups && st == GTOD_OK; ++g) {
      if (g + 1 < n_groups) st = enqueue_group(g + 1);
      if (st == GTOD_OK) st = copy_group(g);
    }
    // drain: every copy queued so far completes before buffers are freed
    (void)hipStreamSynchronize(cs);
    (void)hipStreamSynchronize(xs);
    wr.finish();
    if (wr.failed()) {
      if (st == GTOD_OK || st == GTOD_EIO) {
        st = GTOD_EIO;
        emsg = wr.message();
      }
    }
  }
  for (int fd : {fd_tod, fd_pwv, fd_time})
    if (fd >= 0 && close(fd) != 0 && st == GTOD_OK) {
      st = GTOD_EIO;
      emsg = std::string("close: ") + std::strerror(errno);
    }
  for (int i = 0; i < 2; ++i) {
    for (hipEvent_t e : {computed[i], slab_free[i], piece_ev[i]})
      if (e) (void)hipEventDestroy(e);
    ctx_free(c, tod_slab[i]);
    ctx_free(c, pwv_slab[i]);
  }
  if (host) (void)hipHostFree(host);
  if (st == GTOD_EIO && !emsg.empty()) ctx_fail(c, GTOD_EIO, emsg.c_str());
  if (stats) {
    stats[0] = std::chrono::duration<double>(std::chrono::steady_clock::now() - wall0).count();
    stats[1] = (double)bytes;
    stats[2] = (double)n_groups;
    stats[3] = (double)G;
  }
  return st;
}
