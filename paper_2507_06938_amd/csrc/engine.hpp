// Host-side structures shared by the model and the evaluation engine.
#pragma once
#include <vector>

#include "model.hpp"

struct dl_model {
  dl::ModelDev d{};
  dl::ModelDev* dev = nullptr;  // device copy of d (for kernels)
  std::vector<void*> allocs;
  int64_t m_host[3] = {0, 0, 0};
};

namespace dl {

inline dl_status dev_alloc(std::vector<void*>& list, size_t bytes, void** out,
                           size_t* counter = nullptr) {
  void* p = nullptr;
  if (bytes == 0) bytes = 8;
  if (hipMalloc(&p, bytes) != hipSuccess) return DL_ENOMEM;
  list.push_back(p);
  if (counter) *counter += bytes;
  *out = p;
  return DL_OK;
}

template <typename T>
inline dl_status upload(std::vector<void*>& list, const std::vector<T>& h,
                        const T** out) {
  void* p = nullptr;
  dl_status st = dev_alloc(list, h.size() * sizeof(T), &p);
  if (st != DL_OK) return st;
  if (!h.empty() &&
      hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) !=
          hipSuccess)
    return DL_EHIP;
  *out = (const T*)p;
  return DL_OK;
}


inline void free_all(std::vector<void*>& list) {
  for (void* p : list) (void)hipFree(p);
  list.clear();
}

}  // namespace dl
